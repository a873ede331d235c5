// Tile rasterizer: front-to-back compositing of depth-sorted splats (Eq. 2
// of the paper) and its adjoint.
//
// One 256-lane workgroup (4 wave64) owns a 16x16 tile; each wave owns an 8x8
// quadrant (more compact than 16x4 rows, so a wave's pixels agree more often
// on early termination).  The tile's depth-ordered splat list is streamed
// through LDS in batches; every lane composites its own pixel.  A pixel stops
// before the splat that would take its transmittance below 1e-4; a wave leaves
// the batch loop when its execution mask empties, and the workgroup stops
// loading batches once a block-wide count says every pixel is done.
//
// The adjoint replays the same lists back to front from each pixel's last
// composited splat, recovering T_i = T_{i+1} / (1 - alpha_i) from the saved
// final transmittance instead of storing per-splat state.  Per-splat partial
// derivatives are summed over the wave with DPP row shifts/broadcasts and the
// 9 totals go to HBM with hardware FP32 atomics (one set per wave and splat).
//
// Work items are (view, tile) pairs over every view of the frame.  With
// persistent > 0 a fixed grid takes items from an atomic queue in
// heaviest-list-first order (coarse-to-fine batches mix tiny and full-size
// views, so the tail is what limits a plain launch).
#include "gs_internal.h"

namespace {

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

template <int BATCH>
__global__ void __launch_bounds__(GS_BLOCK) raster_fwd_kernel(RasterArgs a) {
    __shared__ float4 sp0[BATCH], sp1[BATCH], sp2[BATCH];
    __shared__ u32 s_item;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int lx = (w & 1) * 8 + (lane & 7), ly = (w >> 1) * 8 + (lane >> 3);
    u32 item = blockIdx.x;
    for (;;) {
        if (a.queue) {
            __syncthreads();
            if (tid == 0) s_item = atomicAdd(a.queue, 1u);
            __syncthreads();
            item = s_item;
        }
        if (item >= (u32)a.T) break;
        const u32 t = a.order ? a.order[item] : item;
        const int v = find_view(a.views, a.V, t);
        const gs_view_info vi = a.views[v];
        const int lt = (int)t - vi.tile_base;
        const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
        const int px = tx * GS_TILE + lx, py = ty * GS_TILE + ly;
        const bool inside = px < vi.width && py < vi.height;
        const uint2 rg = a.ranges[t];
        const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;

        float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
        u32 last = 0, ncomp = 0;
        bool done = !inside;
        for (u32 b0 = rg.x; b0 < rg.y; b0 += BATCH) {
            if (__syncthreads_count(done) == GS_BLOCK) break;
            const u32 cnt = min((u32)BATCH, rg.y - b0);
            if ((u32)tid < cnt) {
                u32 e = a.inst_entry[b0 + tid];
                if (e >= a.E) e = a.E - 1;   // never taken for a consistent frame
                sp0[tid] = a.splat[3 * (u64)e + 0];
                sp1[tid] = a.splat[3 * (u64)e + 1];
                sp2[tid] = a.splat[3 * (u64)e + 2];
            }
            __syncthreads();
            if (!done) {
                for (u32 k = 0; k < cnt; ++k) {
                    float G, dx, dy;
                    const float raw = splat_raw_alpha(sp0[k], sp1[k], pxc, pyc, G, dx, dy);
                    const float alpha = fminf(raw, GS_ALPHA_MAX);
                    if (alpha < GS_ALPHA_MIN) continue;
                    const float Tn = T * (1.f - alpha);
                    if (Tn < GS_T_MIN) {
                        done = true;
                        break;
                    }
                    const float4 c = sp2[k];
                    const float wgt = alpha * T;
                    C0 = fmaf(c.x, wgt, C0);
                    C1 = fmaf(c.y, wgt, C1);
                    C2 = fmaf(c.z, wgt, C2);
                    T = Tn;
                    last = b0 - rg.x + k + 1;
                    ++ncomp;
                }
            }
        }
        if (inside) {
            const int64_t pix = vi.pix_base + (int64_t)py * vi.width + px;
            const int64_t hw = (int64_t)vi.width * vi.height;
            float* img = a.images + 3 * vi.pix_base + (int64_t)py * vi.width + px;
            img[0] = fmaf(T, a.bg0, C0);
            img[hw] = fmaf(T, a.bg1, C1);
            img[2 * hw] = fmaf(T, a.bg2, C2);
            a.T_final[pix] = T;
            a.n_contrib[pix] = last;
            a.n_comp[pix] = ncomp;
        }
        if (!a.queue) break;
    }
}

template <int BATCH>
__global__ void __launch_bounds__(GS_BLOCK) raster_bwd_kernel(RasterArgs a) {
    __shared__ float4 sp0[BATCH], sp1[BATCH], sp2[BATCH];
    __shared__ u32 se[BATCH];
    __shared__ u32 s_item, s_max;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int lx = (w & 1) * 8 + (lane & 7), ly = (w >> 1) * 8 + (lane >> 3);
    u32 item = blockIdx.x;
    for (;;) {
        if (a.queue) {
            __syncthreads();
            if (tid == 0) s_item = atomicAdd(a.queue, 1u);
            __syncthreads();
            item = s_item;
        }
        if (item >= (u32)a.T) break;
        const u32 t = a.order ? a.order[item] : item;
        const int v = find_view(a.views, a.V, t);
        const gs_view_info vi = a.views[v];
        const int lt = (int)t - vi.tile_base;
        const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
        const int px = tx * GS_TILE + lx, py = ty * GS_TILE + ly;
        const bool inside = px < vi.width && py < vi.height;
        const uint2 rg = a.ranges[t];
        const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;

        float T = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
        u32 last = 0;
        if (inside) {
            const int64_t pix = vi.pix_base + (int64_t)py * vi.width + px;
            const int64_t hw = (int64_t)vi.width * vi.height;
            const float* d = a.dL + 3 * vi.pix_base + (int64_t)py * vi.width + px;
            T = a.T_final[pix];
            last = a.n_contrib[pix];
            g0 = d[0];
            g1 = d[hw];
            g2 = d[2 * hw];
        }
        // colour behind the current splat, background included
        float S0 = T * a.bg0, S1 = T * a.bg1, S2 = T * a.bg2;
        __syncthreads();
        if (tid == 0) s_max = 0;
        __syncthreads();
        if (last) atomicMax(&s_max, last);
        __syncthreads();
        const u32 maxlast = s_max;

        for (int bi = (int)((maxlast + BATCH - 1) / BATCH) - 1; bi >= 0; --bi) {
            const u32 b0 = rg.x + (u32)bi * BATCH;
            const u32 cnt = min((u32)BATCH, maxlast - (u32)bi * BATCH);
            __syncthreads();
            if ((u32)tid < cnt) {
                u32 e = a.inst_entry[b0 + tid];
                if (e >= a.E) e = a.E - 1;   // never taken for a consistent frame
                se[tid] = e;
                sp0[tid] = a.splat[3 * (u64)e + 0];
                sp1[tid] = a.splat[3 * (u64)e + 1];
                sp2[tid] = a.splat[3 * (u64)e + 2];
            }
            __syncthreads();
            for (int k = (int)cnt - 1; k >= 0; --k) {
                const u32 rel = (u32)bi * BATCH + (u32)k;
                float gm0 = 0.f, gm1 = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, gop = 0.f;
                float gr0 = 0.f, gr1 = 0.f, gr2 = 0.f;
                bool contrib = false;
                if (rel < last) {
                    const float4 p1 = sp1[k];
                    float G, dx, dy;
                    const float raw = splat_raw_alpha(sp0[k], p1, pxc, pyc, G, dx, dy);
                    const float alpha = fminf(raw, GS_ALPHA_MAX);
                    if (alpha >= GS_ALPHA_MIN) {
                        contrib = true;
                        const float4 c = sp2[k];
                        const float inv = __builtin_amdgcn_rcpf(1.f - alpha);
                        const float Ti = T * inv;
                        const float wgt = alpha * Ti;
                        gr0 = wgt * g0;
                        gr1 = wgt * g1;
                        gr2 = wgt * g2;
                        const float cd = fmaf(c.x, g0, fmaf(c.y, g1, c.z * g2));
                        const float sd = fmaf(S0, g0, fmaf(S1, g1, S2 * g2));
                        const float dalpha = cd * Ti - sd * inv;
                        S0 = fmaf(c.x, wgt, S0);
                        S1 = fmaf(c.y, wgt, S1);
                        S2 = fmaf(c.z, wgt, S2);
                        T = Ti;
                        if (raw <= GS_ALPHA_MAX) {
                            gop = dalpha * G;
                            const float gG = gop * p1.w;   // dL/dG * G
                            gm0 = gG * fmaf(p1.x, dx, p1.y * dy);
                            gm1 = gG * fmaf(p1.y, dx, p1.z * dy);
                            ga = -0.5f * gG * dx * dx;
                            gb = -gG * dx * dy;
                            gc = -0.5f * gG * dy * dy;
                        }
                    }
                }
                if (__ballot(contrib) == 0) continue;
                gm0 = wave_sum_lane63(gm0);
                gm1 = wave_sum_lane63(gm1);
                ga = wave_sum_lane63(ga);
                gb = wave_sum_lane63(gb);
                gc = wave_sum_lane63(gc);
                gop = wave_sum_lane63(gop);
                gr0 = wave_sum_lane63(gr0);
                gr1 = wave_sum_lane63(gr1);
                gr2 = wave_sum_lane63(gr2);
                if (lane == 63) {
                    float* dst = a.splat_grad + 9 * (u64)se[k];
                    unsafeAtomicAdd(dst + 0, gm0);
                    unsafeAtomicAdd(dst + 1, gm1);
                    unsafeAtomicAdd(dst + 2, ga);
                    unsafeAtomicAdd(dst + 3, gb);
                    unsafeAtomicAdd(dst + 4, gc);
                    unsafeAtomicAdd(dst + 5, gop);
                    unsafeAtomicAdd(dst + 6, gr0);
                    unsafeAtomicAdd(dst + 7, gr1);
                    unsafeAtomicAdd(dst + 8, gr2);
                }
            }
        }
        if (!a.queue) break;
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
        case 64: raster_fwd_kernel<64><<<grid, GS_BLOCK, 0, s>>>(a); break;
        case 128: raster_fwd_kernel<128><<<grid, GS_BLOCK, 0, s>>>(a); break;
        default: raster_fwd_kernel<256><<<grid, GS_BLOCK, 0, s>>>(a); break;
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
        case 64: raster_bwd_kernel<64><<<grid, GS_BLOCK, 0, s>>>(a); break;
        case 128: raster_bwd_kernel<128><<<grid, GS_BLOCK, 0, s>>>(a); break;
        default: raster_bwd_kernel<256><<<grid, GS_BLOCK, 0, s>>>(a); break;
    }
    return gs_check_launch("raster_bwd");
}
