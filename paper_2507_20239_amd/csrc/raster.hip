// Tile rasterizer: front-to-back compositing of depth-sorted splats (Eq. 2
// of the paper) and its adjoint.
//
// One wave64 owns a 16x16 tile and each lane a 2x2 pixel quad (lanes form an
// 8x8 grid of quads).  The tile's depth-ordered splat list is streamed
// through LDS in batches (the lanes load one splat each, then every lane reads
// the batch back with uniform, broadcast LDS loads) and each lane composites
// its four pixels.  A pixel stops before the splat that would take its
// transmittance below 1e-4; the wave leaves the list as soon as a ballot over
// its lanes finds no live pixel.
//
// The adjoint replays the same lists back to front from each pixel's last
// composited splat, recovering T_i = T_{i+1} / (1 - alpha_i) from the saved
// final transmittance instead of storing per-splat state.  Each lane sums
// the partial derivatives of its four pixels, the wave reduces the nine sums
// with DPP row shifts and broadcasts, and one lane adds them to HBM with
// hardware FP32 atomics: one set of atomics per (splat, tile).  Owning a whole
// tile with one wave is what keeps both the reductions and the atomics at one
// per (splat, tile) instead of one per (splat, wave).
//
// Work items are (view, tile) pairs over every view of the frame.  With
// persistent > 0 a fixed grid of waves takes items from an atomic queue in
// heaviest-list-first order (coarse-to-fine batches mix tiny and full-size
// views, so the tail is what limits a plain launch).
#include "gs_internal.h"

namespace {

constexpr int PIX = 4;   // pixels per lane (2x2 quad)

struct RasterArgs {
    const float4* splat;       // [E][3]
    const u32* inst_entry;     // sorted instance -> entry id
    const uint2* ranges;       // [T]
    const gs_view_info* views;
    int V;
    int T;
    u32 E;
    const u32* order;          // heavy-first tile order (persistent mode) or null
    u32* queue;                // work counter (persistent mode) or null
    float bg0, bg1, bg2;
    // forward
    float* images;
    float* T_final;
    u32* n_contrib;
    u32* n_comp;
    // backward
    const float* dL;
    float* splat_grad;
};

__device__ __forceinline__ int find_view(const gs_view_info* views, int V, u32 t) {
    int v = 0;
    while (v + 1 < V && (int)t >= views[v + 1].tile_base) ++v;
    return v;
}

// Next work item of this wave: the block index, or a queue ticket.
__device__ __forceinline__ u32 next_item(const RasterArgs& a, u32 item, bool first) {
    if (!a.queue) return first ? blockIdx.x : (u32)a.T;
    u32 t = 0;
    if (threadIdx.x == 0) t = atomicAdd(a.queue, 1u);
    return __shfl(t, 0, 64);
}

struct TileCoords {
    gs_view_info vi;
    uint2 rg;
    int px0, py0;   // top-left pixel of this lane's quad
};

__device__ __forceinline__ TileCoords tile_coords(const RasterArgs& a, u32 t) {
    TileCoords c;
    const int v = find_view(a.views, a.V, t);
    c.vi = a.views[v];
    const int lt = (int)t - c.vi.tile_base;
    const int tx = lt % c.vi.tiles_x, ty = lt / c.vi.tiles_x;
    const int lane = threadIdx.x;
    c.px0 = tx * GS_TILE + 2 * (lane & 7);
    c.py0 = ty * GS_TILE + 2 * (lane >> 3);
    c.rg = a.ranges[t];
    return c;
}

template <int BATCH>
__device__ __forceinline__ void load_batch(const RasterArgs& a, u32 b0, u32 cnt, float4* sp0,
                                           float4* sp1, float4* sp2, u32* se) {
    for (u32 j = threadIdx.x; j < cnt; j += 64) {
        u32 e = a.inst_entry[b0 + j];
        if (e >= a.E) e = a.E - 1;   // never taken for a consistent frame
        sp0[j] = a.splat[3 * (u64)e + 0];
        sp1[j] = a.splat[3 * (u64)e + 1];
        sp2[j] = a.splat[3 * (u64)e + 2];
        if (se) se[j] = e;
    }
}

template <int BATCH>
__global__ void __launch_bounds__(64) raster_fwd_kernel(RasterArgs a) {
    __shared__ float4 sp0[BATCH], sp1[BATCH], sp2[BATCH];
    for (u32 item = next_item(a, 0, true); item < (u32)a.T; item = next_item(a, item, false)) {
        const u32 t = a.order ? a.order[item] : item;
        const TileCoords tc = tile_coords(a, t);
        float pxc[PIX], pyc[PIX], T[PIX], C0[PIX], C1[PIX], C2[PIX];
        u32 last[PIX], ncomp[PIX];
        bool done[PIX];
#pragma unroll
        for (int i = 0; i < PIX; ++i) {
            const int px = tc.px0 + (i & 1), py = tc.py0 + (i >> 1);
            pxc[i] = (float)px + 0.5f;
            pyc[i] = (float)py + 0.5f;
            T[i] = 1.f;
            C0[i] = C1[i] = C2[i] = 0.f;
            last[i] = 0;
            ncomp[i] = 0;
            done[i] = !(px < tc.vi.width && py < tc.vi.height);
        }
        for (u32 b0 = tc.rg.x; b0 < tc.rg.y; b0 += BATCH) {
            if (__ballot(!(done[0] && done[1] && done[2] && done[3])) == 0) break;
            const u32 cnt = min((u32)BATCH, tc.rg.y - b0);
            __syncthreads();
            load_batch<BATCH>(a, b0, cnt, sp0, sp1, sp2, nullptr);
            __syncthreads();
            for (u32 k = 0; k < cnt; ++k) {
                const float4 p0 = sp0[k], p1 = sp1[k], c = sp2[k];
                const u32 idx = b0 - tc.rg.x + k + 1;
                Quad q;
                quad_setup(p0, p1, pxc[0], pyc[0], q);
                bool live = false;
#pragma unroll
                for (int i = 0; i < PIX; ++i) {
                    const float alpha = fminf(p1.w * quad_G(p1.x, q, i), GS_ALPHA_MAX);
                    bool take = !done[i] && alpha >= GS_ALPHA_MIN;
                    const float Tn = T[i] * (1.f - alpha);
                    const bool stop = take && Tn < GS_T_MIN;
                    done[i] = done[i] || stop;
                    take = take && !stop;
                    const float wgt = take ? alpha * T[i] : 0.f;
                    C0[i] = fmaf(c.x, wgt, C0[i]);
                    C1[i] = fmaf(c.y, wgt, C1[i]);
                    C2[i] = fmaf(c.z, wgt, C2[i]);
                    T[i] = take ? Tn : T[i];
                    last[i] = take ? idx : last[i];
                    ncomp[i] += take ? 1u : 0u;
                    live = live || !done[i];
                }
                if (__ballot(live) == 0) break;
            }
        }
        const int64_t hw = (int64_t)tc.vi.width * tc.vi.height;
#pragma unroll
        for (int i = 0; i < PIX; ++i) {
            const int px = tc.px0 + (i & 1), py = tc.py0 + (i >> 1);
            if (px < tc.vi.width && py < tc.vi.height) {
                const int64_t off = (int64_t)py * tc.vi.width + px;
                float* img = a.images + 3 * tc.vi.pix_base + off;
                img[0] = fmaf(T[i], a.bg0, C0[i]);
                img[hw] = fmaf(T[i], a.bg1, C1[i]);
                img[2 * hw] = fmaf(T[i], a.bg2, C2[i]);
                a.T_final[tc.vi.pix_base + off] = T[i];
                a.n_contrib[tc.vi.pix_base + off] = last[i];
                a.n_comp[tc.vi.pix_base + off] = ncomp[i];
            }
        }
    }
}

template <int BATCH>
__global__ void __launch_bounds__(64) raster_bwd_kernel(RasterArgs a) {
    __shared__ float4 sp0[BATCH], sp1[BATCH], sp2[BATCH];
    __shared__ u32 se[BATCH];
    const int lane = threadIdx.x;
    // factor of each reduced value (lane l holds value l): fa * o + fb
    const float fa = lane < 2 ? 1.f / GS_KAPPA : (lane == 2 || lane == 4) ? -0.5f : lane == 3 ? -1.f : 0.f;
    const float fb = (lane >= 5 && lane < 9) ? 1.f : 0.f;
    for (u32 item = next_item(a, 0, true); item < (u32)a.T; item = next_item(a, item, false)) {
        const u32 t = a.order ? a.order[item] : item;
        const TileCoords tc = tile_coords(a, t);
        const int64_t hw = (int64_t)tc.vi.width * tc.vi.height;
        float pxc[PIX], pyc[PIX], T[PIX], g0[PIX], g1[PIX], g2[PIX], sd[PIX];
        u32 last[PIX];
        u32 mlast = 0;
#pragma unroll
        for (int i = 0; i < PIX; ++i) {
            const int px = tc.px0 + (i & 1), py = tc.py0 + (i >> 1);
            pxc[i] = (float)px + 0.5f;
            pyc[i] = (float)py + 0.5f;
            T[i] = g0[i] = g1[i] = g2[i] = 0.f;
            last[i] = 0;
            if (px < tc.vi.width && py < tc.vi.height) {
                const int64_t off = (int64_t)py * tc.vi.width + px;
                const float* d = a.dL + 3 * tc.vi.pix_base + off;
                T[i] = a.T_final[tc.vi.pix_base + off];
                last[i] = a.n_contrib[tc.vi.pix_base + off];
                g0[i] = d[0];
                g1[i] = d[hw];
                g2[i] = d[2 * hw];
            }
            // dL/dC . (colour behind the current splat), background included
            sd[i] = T[i] * fmaf(a.bg0, g0[i], fmaf(a.bg1, g1[i], a.bg2 * g2[i]));
            mlast = max(mlast, last[i]);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mlast = max(mlast, (u32)__shfl_xor((int)mlast, off, 64));

        for (int bi = (int)((mlast + BATCH - 1) / BATCH) - 1; bi >= 0; --bi) {
            const u32 b0 = tc.rg.x + (u32)bi * BATCH;
            const u32 cnt = min((u32)BATCH, mlast - (u32)bi * BATCH);
            __syncthreads();
            load_batch<BATCH>(a, b0, cnt, sp0, sp1, sp2, se);
            __syncthreads();
            for (int k = (int)cnt - 1; k >= 0; --k) {
                const u32 rel = (u32)bi * BATCH + (u32)k;
                const float4 p0 = sp0[k], p1 = sp1[k], c = sp2[k];
                Quad q;
                quad_setup(p0, p1, pxc[0], pyc[0], q);
                // per pixel: go = dL/dalpha * G (zero where the splat did not
                // contribute or alpha was clamped); per lane: colour gradient sums
                float go[PIX];
                float gr0 = 0.f, gr1 = 0.f, gr2 = 0.f;
                bool contrib = false;
#pragma unroll
                for (int i = 0; i < PIX; ++i) {
                    const float G = quad_G(p1.x, q, i);
                    const float raw = p1.w * G;
                    const float alpha = fminf(raw, GS_ALPHA_MAX);
                    const bool use = rel < last[i] && alpha >= GS_ALPHA_MIN;
                    contrib = contrib || use;
                    // T_i = T_{i+1} / (1 - alpha_i).  The hardware reciprocal is
                    // within 1 ulp but biased, and the bias compounds over a long
                    // back-to-front walk; one Newton step leaves an unbiased error
                    // of about half an ulp.
                    const float om = 1.f - alpha;
                    float inv = __builtin_amdgcn_rcpf(om);
                    inv = fmaf(fmaf(-om, inv, 1.f), inv, inv);
                    const float Ti = T[i] * inv;
                    const float wgt = use ? alpha * Ti : 0.f;
                    const float cd = fmaf(c.x, g0[i], fmaf(c.y, g1[i], c.z * g2[i]));
                    // dL/dalpha = (c . g) T_i - (g . colour behind) / (1 - alpha)
                    const float dalpha = fmaf(cd, Ti, -sd[i] * inv);
                    sd[i] = fmaf(cd, wgt, sd[i]);
                    T[i] = use ? Ti : T[i];
                    gr0 = fmaf(wgt, g0[i], gr0);
                    gr1 = fmaf(wgt, g1[i], gr1);
                    gr2 = fmaf(wgt, g2[i], gr2);
                    go[i] = (use && raw <= GS_ALPHA_MAX) ? dalpha * G : 0.f;
                }
                if (__ballot(contrib) == 0) continue;
                // lane moments of go over the quad: sum go (1, dx, dy, dx^2, dx dy, dy^2),
                // factored by column (pixels 0, 2 | 1, 3) and row (0, 1 | 2, 3)
                const float A0 = go[0] + go[2], A1 = go[1] + go[3];
                const float B0 = go[0] + go[1], B1 = go[2] + go[3];
                float gop = A0 + A1;
                float sx = fmaf(q.dx[0], A0, q.dx[1] * A1);
                float sy = fmaf(q.dy[0], B0, q.dy[1] * B1);
                float sxx = fmaf(q.dx[0] * q.dx[0], A0, (q.dx[1] * q.dx[1]) * A1);
                float syy = fmaf(q.dy[0] * q.dy[0], B0, (q.dy[1] * q.dy[1]) * B1);
                float sxy = fmaf(q.dx[0], fmaf(go[0], q.dy[0], go[2] * q.dy[1]),
                                 q.dx[1] * fmaf(go[1], q.dy[0], go[3] * q.dy[1]));
                // With w = dL/dalpha o G:  dL/dmean = sum w Q d,
                // dL/d(a, b, c) = -sum w (dx^2/2, dx dy, dy^2/2), dL/do = sum dL/dalpha G;
                // Q = L L^T / kappa from the stored Cholesky factor.  Q is applied
                // to the lane sums before the reduction (it is linear), the per-value
                // factors of o after it, and lanes 0..8 then add the nine totals
                // with a single 9-lane atomic instruction, which the memory system
                // coalesces into one request per cache line.
                const float qa = p1.x * p1.x, qb = p1.x * p1.y, qc = fmaf(p1.y, p1.y, p1.z * p1.z);
                float v[9];
                v[0] = fmaf(qa, sx, qb * sy);
                v[1] = fmaf(qb, sx, qc * sy);
                v[2] = sxx;
                v[3] = sxy;
                v[4] = syy;
                v[5] = gop;
                v[6] = gr0;
                v[7] = gr1;
                v[8] = gr2;
                const float val = wave_reduce9(v, lane) * fmaf(p1.w, fa, fb);
                if (lane < 9) unsafeAtomicAdd(a.splat_grad + 9 * (u64)se[k] + lane, val);
            }
        }
    }
}

RasterArgs make_args(gs_frame* f, const gs_raster_opts* o) {
    RasterArgs a;
    a.splat = f->splat;
    a.inst_entry = f->ivals[f->isorted];
    a.ranges = f->ranges;
    a.views = f->d_views;
    a.V = f->V;
    a.T = f->T;
    a.E = (u32)f->E;
    a.order = nullptr;
    a.queue = nullptr;
    a.bg0 = o->bg[0];
    a.bg1 = o->bg[1];
    a.bg2 = o->bg[2];
    a.images = nullptr;
    a.T_final = f->T_final;
    a.n_contrib = f->n_contrib;
    a.n_comp = f->n_comp;
    a.dL = nullptr;
    a.splat_grad = f->splat_grad;
    return a;
}

gs_status grid_for(gs_frame* f, const gs_raster_opts* o, RasterArgs& a, int queue_slot,
                   hipStream_t s, unsigned& grid) {
    if (o->persistent_blocks > 0) {
        GS_TRY(gs_fill_u32(f->counters + queue_slot, 0u, 1, s));
        a.queue = f->counters + queue_slot;
        a.order = f->tvals[f->tsorted];
        grid = (unsigned)o->persistent_blocks;
    } else {
        grid = (unsigned)f->T;
    }
    return GS_OK;
}

}  // namespace

gs_status gs_launch_raster_fwd(gs_frame* f, const gs_raster_opts* o, float* images,
                               hipStream_t s) {
    if (f->T == 0) return GS_OK;
    RasterArgs a = make_args(f, o);
    a.images = images;
    unsigned grid;
    GS_TRY(grid_for(f, o, a, 3, s, grid));
    switch (o->raster_batch) {
        case 64: raster_fwd_kernel<64><<<grid, 64, 0, s>>>(a); break;
        case 256: raster_fwd_kernel<256><<<grid, 64, 0, s>>>(a); break;
        default: raster_fwd_kernel<128><<<grid, 64, 0, s>>>(a); break;
    }
    return gs_check_launch("raster_fwd");
}

gs_status gs_launch_raster_bwd(gs_frame* f, const gs_raster_opts* o, const float* dL,
                               hipStream_t s) {
    if (f->T == 0) return GS_OK;
    RasterArgs a = make_args(f, o);
    a.dL = dL;
    unsigned grid;
    GS_TRY(grid_for(f, o, a, 4, s, grid));
    switch (o->raster_batch) {
        case 64: raster_bwd_kernel<64><<<grid, 64, 0, s>>>(a); break;
        case 256: raster_bwd_kernel<256><<<grid, 64, 0, s>>>(a); break;
        default: raster_bwd_kernel<128><<<grid, 64, 0, s>>>(a); break;
    }
    return gs_check_launch("raster_bwd");
}
