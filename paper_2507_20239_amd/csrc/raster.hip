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
// through an LDS transpose, and nine lanes add them to HBM with one hardware
// FP32 atomic instruction: one set of atomics per (splat, tile).  Owning a
// whole tile with one wave is what keeps both the reductions and the atomics
// at one per (splat, tile) instead of one per (splat, wave).
//
// Work items are (view, tile) pairs over every view of the frame.  With
// persistent > 0 a fixed grid of waves takes items from an atomic queue in
// heaviest-list-first order (coarse-to-fine batches mix tiny and full-size
// views, so the tail is what limits a plain launch).
//
// A small frame (a coarse level of the coarse-to-fine schedule, or a tiny
// view) has at most a couple of tiles per SIMD, and one wave per tile then
// runs every splat step at a single wave's dependent latency.  Such frames
// take one pixel per lane instead: four waves per tile, each owning an 8x8
// quarter and walking the tile's whole list.  Each pixel's arithmetic is the
// same in both layouts (the single-pixel path repeats the quad's operations
// for its pixel), so images, transmittance and walk lengths are bit-identical;
// the adjoint then adds four partial sums per (splat, tile) instead of one.
#include "gs_internal.h"

namespace {

// Frames with fewer tiles than this take one pixel per lane (plain grid).
constexpr int PIXEL_LANE_MAX_TILES = 2048;

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
    const float* l1_target;    // with the L1 term of Eq. 3 fused: targets, or null
    float* l1_grad;
    float* l1_loss;
    float l1_scale;
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
__device__ __forceinline__ u32 next_item(const RasterArgs& a, u32 n_items, bool first) {
    if (!a.queue) return first ? blockIdx.x : n_items;
    u32 t = 0;
    if (threadIdx.x == 0) t = atomicAdd(a.queue, 1u);
    return __builtin_amdgcn_readfirstlane(t);
}

constexpr int RED_STRIDE = 68;   // floats per row of the reduction transpose buffer

// Order this wave's LDS accesses before and after the call (compiler-level:
// a single wave's LDS operations already execute in program order).
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane layout.  PIXQ = 4: lane l owns the 2x2 quad whose top-left pixel is
// (16 tx + 2 (l % 8), 16 ty + 2 (l / 8)); grouped by quadrant (the forward),
// lanes 16 q .. 16 q + 15 own quadrant q, the 8x8 pixels at (16 tx + 8 (q % 2),
// 16 ty + 8 (q / 2)), lane 16 q + j the quad at (2 (j % 4), 2 (j / 4)) of it.
// PIXQ = 1: work item 4 t + q is quarter (quadrant) q of tile t, and lane l
// owns pixel (l % 8, l / 8) of it.  Either way a lane's pixels lie in one quad
// with top-left pixel (qx, qy); its pixel i is (qx + i % 2, qy + i / 2), for
// i < 4 (quads) or i = pi (one pixel).
struct TileCoords {
    gs_view_info vi;
    uint2 rg;
    int tx, ty;     // tile of the view
    int q;          // the quadrant of the lane's pixels (grouped quads, one pixel per lane)
    int qx, qy;     // top-left pixel of the lane's quad
    int pi;         // one pixel per lane: the lane's pixel within its quad
};

template <int PIXQ, bool GROUPED>
__device__ __forceinline__ TileCoords tile_coords(const RasterArgs& a, u32 t, u32 quarter) {
    TileCoords c;
    const int v = find_view(a.views, a.V, t);
    c.vi = a.views[v];
    const int lt = (int)t - c.vi.tile_base;
    c.tx = lt % c.vi.tiles_x;
    c.ty = lt / c.vi.tiles_x;
    const int lane = threadIdx.x;
    if (PIXQ == 4 && GROUPED) {
        c.q = lane >> 4;
        const int j = lane & 15;
        c.qx = c.tx * GS_TILE + 8 * (c.q & 1) + 2 * (j & 3);
        c.qy = c.ty * GS_TILE + 8 * (c.q >> 1) + 2 * (j >> 2);
        c.pi = 0;
    } else if (PIXQ == 4) {
        c.q = 0;
        c.qx = c.tx * GS_TILE + 2 * (lane & 7);
        c.qy = c.ty * GS_TILE + 2 * (lane >> 3);
        c.pi = 0;
    } else {
        c.q = (int)quarter;
        const int px = c.tx * GS_TILE + 8 * (int)(quarter & 1u) + (lane & 7);
        const int py = c.ty * GS_TILE + 8 * (int)(quarter >> 1) + (lane >> 3);
        c.qx = px & ~1;
        c.qy = py & ~1;
        c.pi = (px & 1) | ((py & 1) << 1);
    }
    c.rg = a.ranges[t];
    return c;
}

// Pixel i of the lane, as an index into its quad.
template <int PIXQ>
__device__ __forceinline__ int quad_pixel(const TileCoords& c, int i) {
    return PIXQ == 4 ? i : c.pi;
}

// A splat's Gaussian at the lane's pixels.  The quad form evaluates all four
// pixels of the quad; the single-pixel form repeats the quad's operations for
// the lane's one pixel (same operands, same order), so both give bit-identical
// values.
template <int PIXQ>
struct LaneGeom;

template <>
struct LaneGeom<4> {
    Quad q;
    __device__ __forceinline__ void setup(float4 p0, float4 p1, float qxc, float qyc, int) {
        quad_setup(p0, p1, qxc, qyc, q);
    }
    __device__ __forceinline__ float G(int i) const { return quad_G(q, i); }
};

template <>
struct LaneGeom<1> {
    float dx, dy, u, vv;
    // The quad's steps for pixel pi: each "+ step" of the quad is taken as
    // fma(o, step, x) with o = 1 or 0 the lane's (constant) pixel offset,
    // which rounds like x + step for o = 1 and returns x for o = 0, one
    // instruction instead of an add and a select.
    __device__ __forceinline__ void setup(float4 p0, float4 p1, float qxc, float qyc, int pi) {
        const float ox = (pi & 1) ? 1.f : 0.f, oy = (pi & 2) ? 1.f : 0.f;
        const float dx0 = (qxc - p0.x) - p0.z;
        const float dy0 = (qyc - p0.y) - p0.w;
        dx = dx0 + ox;
        dy = dy0 + oy;
        const float u0 = fmaf(p1.x, dx0, p1.y * dy0);
        u = fmaf(oy, p1.y, fmaf(ox, p1.x, u0));
        const float v = fmaf(oy, p1.z, p1.z * dy0);
        vv = v * v;
    }
    __device__ __forceinline__ float G(int) const {
        return __builtin_amdgcn_exp2f(-fmaf(u, u, vv));
    }
};

// One batch of a tile's list in LDS: the splat records (the fourth component
// of the colour record, unused in HBM, carries the entry id; record BATCH is
// all zeros, so alpha is 0 at every pixel and a step on it changes nothing)
// and NQ quadrant lists: per quadrant, the batch indices of the splats whose
// footprint meets it, in list order, padded with BATCH to the longest (one
// slot more: the walk reads the next index ahead of its use).  NQ = 4: the
// grouped quads of the forward; NQ = 1: a quarter's wave (one pixel per
// lane); NQ = 0: the whole batch in order.
template <int BATCH, int NQ>
struct Stage {
    float4 sp0[BATCH + 1], sp1[BATCH + 1], sp2[BATCH + 1];
    unsigned short sub[NQ > 0 ? NQ : 1][NQ > 0 ? BATCH + 2 : 1];
};

template <int BATCH, int NQ>
__device__ __forceinline__ void zero_record(Stage<BATCH, NQ>& S) {
    if (threadIdx.x == 0) {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        S.sp0[BATCH] = z;
        S.sp1[BATCH] = z;
        S.sp2[BATCH] = z;
    }
}

// Stage splats [b0, b0 + cnt) of the sorted instance list and build the
// quadrant lists (list q: the splats j < lim[q] whose footprint meets
// quadrant q, or the wave's quadrant tc.q when NQ = 1), from the tile
// culling's ellipse test at half resolution.  A pixel outside every quadrant
// a splat meets has alpha < 1/255 for it, so walking only its quadrant's list
// leaves every pixel's compositing unchanged.  Returns the number of steps:
// the longest list, or cnt when NQ = 0.
template <int BATCH, int NQ>
__device__ __forceinline__ u32 stage_batch(const RasterArgs& a, u32 b0, u32 cnt, const u32* lim,
                                           const TileCoords& tc, Stage<BATCH, NQ>& S) {
    const u32 lane = threadIdx.x;
    u32 n[NQ > 0 ? NQ : 1];
#pragma unroll
    for (int q = 0; q < (NQ > 0 ? NQ : 1); ++q) n[q] = 0;
    for (u32 r = 0; r < cnt; r += 64) {
        const u32 j = r + lane;
        u32 m = 0;
        if (j < cnt) {
            u32 e = a.inst_entry[b0 + j];
            if (e >= a.E) e = a.E - 1;   // never taken for a consistent frame
            const float4 p0 = a.splat[3 * (u64)e + 0];
            const float4 p1 = a.splat[3 * (u64)e + 1];
            float4 c = a.splat[3 * (u64)e + 2];
            c.w = __uint_as_float(e);
            S.sp0[j] = p0;
            S.sp1[j] = p1;
            S.sp2[j] = c;
            if (NQ > 0) m = quadrant_mask(footprint_rows(p0, p1), tc.tx, tc.ty);
            if (NQ == 1) m >>= tc.q;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const bool in = ((m >> q) & 1u) != 0 && j < lim[q];
            const u64 bal = __ballot(in);
            if (in) S.sub[q][n[q] + popc_below(bal)] = (unsigned short)j;
            n[q] += (u32)__popcll(bal);
        }
    }
    if (NQ == 0) return cnt;
    u32 nmax = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) nmax = max(nmax, n[q]);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        for (u32 s = n[q] + lane; s <= nmax; s += 64) S.sub[q][s] = (unsigned short)BATCH;
    return nmax;
}

// Some pixel of the lane still composites (T > 0).  Signed-integer order of
// the bit patterns agrees with the float order on the sign and on positive
// values, so one integer max decides it.
template <int PIXQ>
__device__ __forceinline__ bool any_live(const float* T) {
    if constexpr (PIXQ == 1) {
        return __float_as_int(T[0]) > 0;
    } else {
        const int m = max(max(__float_as_int(T[0]), __float_as_int(T[1])),
                          max(__float_as_int(T[2]), __float_as_int(T[3])));
        return m > 0;
    }
}

template <int BATCH, bool COUNT, int PIXQ>
__global__ void __launch_bounds__(64) raster_fwd_kernel(RasterArgs a) {
    constexpr int NQ = PIXQ == 4 ? 4 : 1;
    __shared__ Stage<BATCH, NQ> S;
    zero_record(S);
    const u32 n_items = PIXQ == 4 ? (u32)a.T : 4u * (u32)a.T;
    for (u32 item = next_item(a, n_items, true); item < n_items;
         item = next_item(a, n_items, false)) {
        const u32 it = __builtin_amdgcn_readfirstlane(a.order ? a.order[item] : item);
        const u32 t = PIXQ == 4 ? it : it >> 2;
        if (t >= (u32)a.T) continue;   // never taken for an order the binning built
        const TileCoords tc = tile_coords<PIXQ, true>(a, t, it & 3u);
        const float qxc = (float)tc.qx + 0.5f, qyc = (float)tc.qy + 0.5f;
        // T < 0 marks a finished pixel, with |T| its final transmittance
        // (pixels outside the image start finished); the sign replaces a
        // per-pixel flag and keeps the state update at two selects.
        float T[PIXQ], C0[PIXQ], C1[PIXQ], C2[PIXQ];
        u32 last[PIXQ], ncomp[PIXQ];
#pragma unroll
        for (int i = 0; i < PIXQ; ++i) {
            const int qp = quad_pixel<PIXQ>(tc, i);
            const int px = tc.qx + (qp & 1), py = tc.qy + (qp >> 1);
            T[i] = (px < tc.vi.width && py < tc.vi.height) ? 1.f : -1.f;
            C0[i] = C1[i] = C2[i] = 0.f;
            last[i] = 0;
            ncomp[i] = 0;
        }
        // each lane walks the list of its quadrant (the four 16-lane groups of a
        // quad wave walk four lists side by side, as many steps as the longest)
        const unsigned short* my = S.sub[PIXQ == 4 ? tc.q : 0];
        for (u32 b0 = tc.rg.x; b0 < tc.rg.y; b0 += BATCH) {
            const u64 live = __ballot(any_live<PIXQ>(T));
            if (live == 0) break;
            const u32 cnt = min((u32)BATCH, tc.rg.y - b0);
            // a quadrant whose pixels have all finished needs no list
            u32 lim[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                lim[q] = PIXQ == 1 || ((live >> (16 * q)) & 0xffffull) != 0 ? cnt : 0u;
            __syncthreads();
            const u32 n = stage_batch<BATCH, NQ>(a, b0, cnt, lim, tc, S);
            __syncthreads();
            // idx: the list position + 1
            const u32 base = b0 - tc.rg.x + 1;
            u32 kn = my[0];
            for (u32 s = 0; s < n; ++s) {
                const u32 k = kn;
                kn = my[s + 1];
                const float4 p0 = S.sp0[k], p1 = S.sp1[k], c = S.sp2[k];
                const u32 idx = base + k;
                LaneGeom<PIXQ> g;
                g.setup(p0, p1, qxc, qyc, tc.pi);
#pragma unroll
                for (int i = 0; i < PIXQ; ++i) {
                    const float alpha = fminf(p1.w * g.G(i), GS_ALPHA_MAX);
                    const bool hit = alpha >= GS_ALPHA_MIN;
                    // T (1 - alpha) with one rounding; a finished pixel has T < 0,
                    // so Tn < 0 and it never takes
                    const float Tn = fmaf(-alpha, T[i], T[i]);
                    const bool take = hit && Tn >= GS_T_MIN;
                    // alpha T as the drop in transmittance
                    const float wgt = take ? T[i] - Tn : 0.f;
                    // a hit that would drop T below the threshold finishes the pixel
                    const float Tkeep = hit ? -fabsf(T[i]) : T[i];
                    T[i] = take ? Tn : Tkeep;
                    C0[i] = fmaf(c.x, wgt, C0[i]);
                    C1[i] = fmaf(c.y, wgt, C1[i]);
                    C2[i] = fmaf(c.z, wgt, C2[i]);
                    last[i] = take ? idx : last[i];
                    if (COUNT) ncomp[i] += take ? 1u : 0u;
                }
                if (__ballot(any_live<PIXQ>(T)) == 0) break;
            }
        }
        const int64_t hw = (int64_t)tc.vi.width * tc.vi.height;
        float l1 = 0.f;   // this lane's share of sum |I - T| (the fused L1 term)
#pragma unroll
        for (int i = 0; i < PIXQ; ++i) {
            const int qp = quad_pixel<PIXQ>(tc, i);
            const int px = tc.qx + (qp & 1), py = tc.qy + (qp >> 1);
            if (px < tc.vi.width && py < tc.vi.height) {
                const int64_t off = (int64_t)py * tc.vi.width + px;
                float* img = a.images + 3 * tc.vi.pix_base + off;
                const float Tf = fabsf(T[i]);
                const float c[3] = {fmaf(Tf, a.bg0, C0[i]), fmaf(Tf, a.bg1, C1[i]),
                                    fmaf(Tf, a.bg2, C2[i])};
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) img[ch * hw] = c[ch];
                if (a.l1_target) {
                    // the L1 term: |I - T| summed, scale * sign(I - T) as the gradient
                    const float* tg = a.l1_target + 3 * tc.vi.pix_base + off;
                    float* gd = a.l1_grad + 3 * tc.vi.pix_base + off;
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        const float d = c[ch] - tg[ch * hw];
                        gd[ch * hw] = d > 0.f ? a.l1_scale : (d < 0.f ? -a.l1_scale : 0.f);
                        l1 += fabsf(d);
                    }
                }
                a.T_final[tc.vi.pix_base + off] = Tf;
                a.n_contrib[tc.vi.pix_base + off] = last[i];
                if (COUNT) a.n_comp[tc.vi.pix_base + off] = ncomp[i];
            }
        }
        if (a.l1_target) {
            // one atomic per work item
            l1 = wave_sum_lane63(l1);
            if (threadIdx.x == 63) unsafeAtomicAdd(a.l1_loss, l1 * a.l1_scale);
        }
    }
}

template <int BATCH, int PIXQ>
__global__ void __launch_bounds__(64) raster_bwd_kernel(RasterArgs a) {
    constexpr int NQ = PIXQ == 4 ? 0 : 1;
    __shared__ Stage<BATCH, NQ> S;
    // transpose buffer of the per-splat reduction: value j of lane l at red[j][l]
    // (rows padded by 16 bytes to spread the 16-byte reads over the banks)
    __shared__ float red[9][RED_STRIDE];
    const int lane = threadIdx.x;
    // lanes 4j .. 4j+3 (j < 9) sum value j; its factor is fa * o + fb
    const int rj = lane >> 2;
    const float fa = rj < 2 ? 1.f / GS_KAPPA : (rj == 2 || rj == 4) ? -0.5f : rj == 3 ? -1.f : 0.f;
    const float fb = (rj >= 5 && rj < 9) ? 1.f : 0.f;
    const u32 n_items = PIXQ == 4 ? (u32)a.T : 4u * (u32)a.T;
    for (u32 item = next_item(a, n_items, true); item < n_items;
         item = next_item(a, n_items, false)) {
        const u32 it = __builtin_amdgcn_readfirstlane(a.order ? a.order[item] : item);
        const u32 t = PIXQ == 4 ? it : it >> 2;
        if (t >= (u32)a.T) continue;   // never taken for an order the binning built
        const TileCoords tc = tile_coords<PIXQ, false>(a, t, it & 3u);
        const float qxc = (float)tc.qx + 0.5f, qyc = (float)tc.qy + 0.5f;
        const int64_t hw = (int64_t)tc.vi.width * tc.vi.height;
        float T[PIXQ], g0[PIXQ], g1[PIXQ], g2[PIXQ], sd[PIXQ];
        u32 last[PIXQ];
        u32 mlast = 0;
#pragma unroll
        for (int i = 0; i < PIXQ; ++i) {
            const int qp = quad_pixel<PIXQ>(tc, i);
            const int px = tc.qx + (qp & 1), py = tc.qy + (qp >> 1);
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
        mlast = __builtin_amdgcn_readfirstlane(mlast);   // uniform: keeps the walk on scalar registers

        for (int bi = (int)((mlast + BATCH - 1) / BATCH) - 1; bi >= 0; --bi) {
            const u32 b0 = tc.rg.x + (u32)bi * BATCH;
            const u32 cnt = min((u32)BATCH, mlast - (u32)bi * BATCH);
            const u32 lim[1] = {cnt};
            __syncthreads();
            const u32 n = stage_batch<BATCH, NQ>(a, b0, cnt, lim, tc, S);
            __syncthreads();
            // back to front over the batch (quads) or the quadrant's list
            u32 kn = 0;
            if constexpr (NQ == 1) kn = S.sub[0][n > 0 ? n - 1 : 0];
            for (int s = (int)n - 1; s >= 0; --s) {
                u32 k = (u32)s;
                if constexpr (NQ == 1) {
                    k = kn;
                    kn = S.sub[0][s > 0 ? s - 1 : 0];
                }
                const u32 rel = (u32)bi * BATCH + k;
                const float4 p0 = S.sp0[k], p1 = S.sp1[k], c = S.sp2[k];
                LaneGeom<PIXQ> g;
                g.setup(p0, p1, qxc, qyc, tc.pi);
                // per pixel: go = dL/dalpha * G (zero where the splat did not
                // contribute or alpha was clamped); per lane: colour gradient sums
                float go[PIXQ];
                float gr0 = 0.f, gr1 = 0.f, gr2 = 0.f;
                bool contrib = false;
#pragma unroll
                for (int i = 0; i < PIXQ; ++i) {
                    const float G = g.G(i);
                    const float raw = p1.w * G;
                    const float alpha = fminf(raw, GS_ALPHA_MAX);
                    const bool use = rel < last[i] && alpha >= GS_ALPHA_MIN;
                    contrib = contrib || use;
                    // an unused splat acts as alpha = 0: the reciprocal below is
                    // then exactly 1, T stays and the weight is 0, with no selects
                    const float au = use ? alpha : 0.f;
                    // T_i = T_{i+1} / (1 - alpha_i).  The hardware reciprocal is
                    // within 1 ulp but biased, and the bias compounds over a long
                    // back-to-front walk; one Newton step leaves an unbiased error
                    // of about half an ulp.
                    const float om = 1.f - au;
                    float inv = __builtin_amdgcn_rcpf(om);
                    inv = fmaf(fmaf(-om, inv, 1.f), inv, inv);
                    const float Ti = T[i] * inv;
                    const float wgt = au * Ti;
                    const float cd = fmaf(c.x, g0[i], fmaf(c.y, g1[i], c.z * g2[i]));
                    // dL/dalpha = (c . g) T_i - (g . colour behind) / (1 - alpha)
                    const float dalpha = fmaf(cd, Ti, -sd[i] * inv);
                    sd[i] = fmaf(cd, wgt, sd[i]);
                    T[i] = Ti;
                    gr0 = fmaf(wgt, g0[i], gr0);
                    gr1 = fmaf(wgt, g1[i], gr1);
                    gr2 = fmaf(wgt, g2[i], gr2);
                    go[i] = (use && raw <= GS_ALPHA_MAX) ? dalpha * G : 0.f;
                }
                if (__ballot(contrib) == 0) continue;
                // lane moments of go over its pixels: sums of go (1, dx, dy, dx^2,
                // dx dy, dy^2), each pixel with its own offsets (an expansion
                // around one pixel would cancel when the others sit next to the
                // splat's centre)
                float gop, sx, sy, sxx, syy, sxy;
                if constexpr (PIXQ == 4) {
                    // factored by column (pixels 0, 2 | 1, 3) and row (0, 1 | 2, 3)
                    const Quad& q = g.q;
                    const float A0 = go[0] + go[2], A1 = go[1] + go[3];
                    const float B0 = go[0] + go[1], B1 = go[2] + go[3];
                    gop = A0 + A1;
                    const float X0 = q.dx[0] * A0, X1 = q.dx[1] * A1;
                    const float Y0 = q.dy[0] * B0, Y1 = q.dy[1] * B1;
                    sx = X0 + X1;
                    sy = Y0 + Y1;
                    sxx = fmaf(q.dx[0], X0, q.dx[1] * X1);
                    syy = fmaf(q.dy[0], Y0, q.dy[1] * Y1);
                    sxy = fmaf(q.dx[0], fmaf(go[0], q.dy[0], go[2] * q.dy[1]),
                               q.dx[1] * fmaf(go[1], q.dy[0], go[3] * q.dy[1]));
                } else {
                    gop = go[0];
                    sx = g.dx * gop;
                    sy = g.dy * gop;
                    sxx = g.dx * sx;
                    syy = g.dy * sy;
                    sxy = g.dx * sy;
                }
                // With w = dL/dalpha o G:  dL/dmean = sum w Q d,
                // dL/d(a, b, c) = -sum w (dx^2/2, dx dy, dy^2/2), dL/do = sum dL/dalpha G;
                // Q = L L^T / kappa from the stored Cholesky factor.  Q is applied
                // to the lane sums before the reduction (it is linear), the per-value
                // factors of o after it.
                const float qa = p1.x * p1.x, qb = p1.x * p1.y, qc = fmaf(p1.y, p1.y, p1.z * p1.z);
                // The nine lane sums go through LDS: every lane writes its row
                // entries, lanes 4j .. 4j+3 read back a quarter of row j each (four
                // 16-byte loads) and two quad DPP adds finish the totals, so lanes
                // 0, 4, .., 32 hold them and add them to HBM with one atomic
                // instruction.  The workgroup is this one wave, whose LDS accesses
                // execute in order; the wavefront fences keep the compiler from
                // moving the accesses across each other.
                red[0][lane] = fmaf(qa, sx, qb * sy);
                red[1][lane] = fmaf(qb, sx, qc * sy);
                red[2][lane] = sxx;
                red[3][lane] = sxy;
                red[4][lane] = syy;
                red[5][lane] = gop;
                red[6][lane] = gr0;
                red[7][lane] = gr1;
                red[8][lane] = gr2;
                wave_sync_lds();
                float tot = 0.f;
                if (rj < 9) {
                    const float4* row = reinterpret_cast<const float4*>(&red[rj][16 * (lane & 3)]);
                    const float4 x0 = row[0], x1 = row[1], x2 = row[2], x3 = row[3];
                    tot = ((x0.x + x0.y) + (x0.z + x0.w)) + ((x1.x + x1.y) + (x1.z + x1.w)) +
                          (((x2.x + x2.y) + (x2.z + x2.w)) + ((x3.x + x3.y) + (x3.z + x3.w)));
                }
                wave_sync_lds();
                tot += dpp_mov_zero<0xB1, 0xF>(tot);   // quad_perm [1,0,3,2]
                tot += dpp_mov_zero<0x4E, 0xF>(tot);   // quad_perm [2,3,0,1]
                if ((lane & 3) == 0 && rj < 9)
                    unsafeAtomicAdd(a.splat_grad + 9 * (u64)__float_as_uint(c.w) + rj,
                                    tot * fmaf(p1.w, fa, fb));
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
    a.l1_target = nullptr;
    a.l1_grad = nullptr;
    a.l1_loss = nullptr;
    a.l1_scale = 0.f;
    a.T_final = f->T_final;
    a.n_contrib = f->n_contrib;
    a.n_comp = f->n_comp;
    a.dL = nullptr;
    a.splat_grad = f->splat_grad;
    return a;
}

// One pixel per lane: forced by GS_RASTER_LANE_PIXELS, else chosen for a small
// frame on the plain grid unless GS_RASTER_LANE_QUADS asks for quads.
bool pixel_lanes(const gs_frame* f, const gs_raster_opts* o) {
    if (o->flags & GS_RASTER_LANE_PIXELS) return true;
    if (o->flags & GS_RASTER_LANE_QUADS) return false;
    return o->persistent_blocks == 0 && f->T < PIXEL_LANE_MAX_TILES;
}

gs_status grid_for(gs_frame* f, const gs_raster_opts* o, RasterArgs& a, int queue_slot,
                   hipStream_t s, bool pixels, unsigned& grid) {
    if (pixels) {
        grid = 4u * (unsigned)f->T;   // four quarter-tile waves per tile (plain grid)
    } else if (o->persistent_blocks > 0) {
        GS_TRY(gs_fill_u32(f->counters + queue_slot, 0u, 1, s));
        a.queue = f->counters + queue_slot;
        a.order = f->tvals[f->tsorted];
        grid = (unsigned)o->persistent_blocks;
    } else {
        grid = (unsigned)f->T;
    }
    return GS_OK;
}

template <int BATCH, int PIXQ>
void launch_fwd(const RasterArgs& a, bool count, unsigned grid, hipStream_t s) {
    if (count) raster_fwd_kernel<BATCH, true, PIXQ><<<grid, 64, 0, s>>>(a);
    else raster_fwd_kernel<BATCH, false, PIXQ><<<grid, 64, 0, s>>>(a);
}

template <int PIXQ>
void launch_fwd_batch(const RasterArgs& a, int batch, bool count, unsigned grid, hipStream_t s) {
    switch (batch) {
        case 128: launch_fwd<128, PIXQ>(a, count, grid, s); break;
        case 256: launch_fwd<256, PIXQ>(a, count, grid, s); break;
        default: launch_fwd<64, PIXQ>(a, count, grid, s); break;
    }
}

template <int PIXQ>
void launch_bwd_batch(const RasterArgs& a, int batch, unsigned grid, hipStream_t s) {
    switch (batch) {
        case 128: raster_bwd_kernel<128, PIXQ><<<grid, 64, 0, s>>>(a); break;
        case 256: raster_bwd_kernel<256, PIXQ><<<grid, 64, 0, s>>>(a); break;
        default: raster_bwd_kernel<64, PIXQ><<<grid, 64, 0, s>>>(a); break;
    }
}

}  // namespace

gs_status gs_launch_raster_fwd(gs_frame* f, const gs_raster_opts* o, float* images,
                               const float* targets, float l1_scale, float* loss, float* dL,
                               hipStream_t s) {
    if (f->T == 0) return GS_OK;
    RasterArgs a = make_args(f, o);
    a.images = images;
    a.l1_target = targets;
    a.l1_grad = dL;
    a.l1_loss = loss;
    a.l1_scale = l1_scale;
    const bool pixels = pixel_lanes(f, o);
    unsigned grid;
    GS_TRY(grid_for(f, o, a, 3, s, pixels, grid));
    const bool count = (o->flags & GS_RASTER_COUNT_COMPOSITED) != 0;
    if (pixels) launch_fwd_batch<1>(a, o->raster_batch, count, grid, s);
    else launch_fwd_batch<4>(a, o->raster_batch, count, grid, s);
    return gs_check_launch("raster_fwd");
}

gs_status gs_launch_raster_bwd(gs_frame* f, const gs_raster_opts* o, const float* dL,
                               hipStream_t s) {
    if (f->T == 0) return GS_OK;
    RasterArgs a = make_args(f, o);
    a.dL = dL;
    const bool pixels = pixel_lanes(f, o);
    unsigned grid;
    GS_TRY(grid_for(f, o, a, 4, s, pixels, grid));
    if (pixels) launch_bwd_batch<1>(a, o->raster_batch, grid, s);
    else launch_bwd_batch<4>(a, o->raster_batch, grid, s);
    return gs_check_launch("raster_bwd");
}
