// Internal declarations shared by the HIP translation units of libgsmi.
// Target: gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsmi.h"

typedef uint32_t u32;
typedef uint64_t u64;

// Rendering constants (FP32 values; the CPU reference uses the same values).
#define GS_ALPHA_MAX 0.99f
#define GS_ALPHA_MIN (1.0f / 255.0f)
#define GS_T_MIN 1e-4f
#define GS_DILATION 0.3f
#define GS_FOV_CLAMP 1.3f
#define GS_FOOTPRINT_INFLATE (1.0 + 1.0 / 1024.0)

#define GS_WAVE 64
#define GS_BLOCK 256

// Per-view constants kept in device memory (32 bytes).
struct gs_view_info {
    int32_t width, height, tiles_x, tiles_y;
    int32_t tile_base;   // first global tile id of the view
    int32_t pad;
    int64_t pix_base;    // first pixel of the view in the per-pixel arrays
};

struct gs_frame {
    int64_t n;           // Gaussians
    int32_t V;           // views
    int64_t E;           // entries = V * n
    int64_t cap;         // instance capacity
    int32_t T;           // tiles over all views
    int64_t P;           // pixels over all views
    gs_view_info views[GS_MAX_VIEWS];
    gs_view_info* d_views;

    // projection
    u32* depth_key;      // [E]
    u32* tiles_touched;  // [E]
    uint2* rect;         // [E]
    float4* splat;       // [E][3]
    // visible-entry compaction
    u32* visible;        // [E] visible entries, in entry order
    u32* inst_off;       // [E] instance offset of each visible entry
    // depth presort of the visible entries: keys (ping-pong) and the second value slot
    u32* dkeys[2];       // [E]
    u32* dvals1;         // [E]
    // instances (ping-pong)
    u32* ikeys[2];       // [cap]
    u32* ivals[2];       // [cap]
    u32* chunk_start;    // [cap / 256 + 1] first entry of each 256-instance chunk
    int isorted;
    uint2* ranges;       // [T]
    // heavy-first tile order for persistent launches
    u32* tkeys[2];       // [T]
    u32* tvals[2];       // [T]
    int tsorted;
    bool heavy_built;    // the last binning built the heavy-first order (tvals[tsorted])
    int32_t tile_bits;   // bits needed for a global tile id
    bool sigma3;         // the last projection binned by 3-sigma squares
    // per pixel
    float* T_final;      // [P]
    u32* n_contrib;      // [P]
    u32* n_comp;         // [P] splats composited per pixel
    // per splat gradient
    float* splat_grad;   // [E][9]
    // counters: [0] visible, [1] instances, [2] overflow, [3] fwd queue, [4] bwd queue,
    // [5] instances kept (min(instances, capacity)), [6] sticky overflow (set by any
    // binning that overflowed, cleared only by the caller)
    u32* counters;
    // sort and scan scratch
    void* sort_scratch;
    u32* scan_part;      // [4 (GS_SCAN_PARTS + 8)] (u32 or u64 partial sums)
};

#define GS_SCAN_PARTS 1024

// ------------------------------------------------------------------------
// Status
// ------------------------------------------------------------------------
gs_status gs_fail(gs_status s, const char* fmt, ...);
gs_status gs_check_launch(const char* what);

#define GS_HIP(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess)                                                       \
            return gs_fail(GS_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_)); \
    } while (0)

#define GS_TRY(x)                        \
    do {                                 \
        gs_status s_ = (x);              \
        if (s_ != GS_OK) return s_;      \
    } while (0)


// ------------------------------------------------------------------------
// Two-launch exclusive scan.  The first launch (gs_scan_reduce) sums each of
// GS_SCAN_PARTS partitions; every workgroup of the second adds up the partial
// sums before its own partition (at most 1024 values, read by 256 threads),
// scans its partition and hands each (index, value, exclusive prefix) to an
// epilogue, which stores the prefix or does more with it (stream compaction,
// chunk starts); the last workgroup hands the grand total to epi.finish.
// ------------------------------------------------------------------------
__device__ __forceinline__ u32 dev_len(const u32* n_dev, u32 n_host) {
    return n_dev ? *n_dev : n_host;
}

__device__ __forceinline__ void chunk_of(u32 n, u32 parts, u32 b, u32& beg, u32& end) {
    u32 chunk = (n + parts - 1) / parts;
    chunk = (chunk + 63u) & ~63u;
    const u64 b0 = (u64)b * chunk;
    beg = b0 < n ? (u32)b0 : n;
    const u64 e0 = (u64)beg + chunk;
    end = e0 < n ? (u32)e0 : n;
}

__device__ __forceinline__ u32 shfl_up_any(u32 x, int d) { return (u32)__shfl_up((int)x, d, 64); }
__device__ __forceinline__ u64 shfl_up_any(u64 x, int d) {
    const u32 lo = (u32)__shfl_up((int)(u32)x, d, 64);
    const u32 hi = (u32)__shfl_up((int)(u32)(x >> 32), d, 64);
    return ((u64)hi << 32) | lo;
}

// Exclusive scan of one value per thread over a 256-thread workgroup (u32 or u64).
template <class V>
__device__ __forceinline__ V block_exclusive_scan(V v, V* lds4, V& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    V x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const V y = shfl_up_any(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds4[w] = x;
    __syncthreads();
    V wbase = 0;
    for (int j = 0; j < w; ++j) wbase += lds4[j];
    total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
    __syncthreads();
    return wbase + x - v;
}

__device__ __forceinline__ u32 scan_in(const u32* in, const u32* gather, u32 i) {
    return gather ? in[gather[i]] : in[i];
}

// This thread's share of the sum of the partition totals before partition b
// (b < GS_SCAN_PARTS): its GS_SCAN_PARTS / GS_BLOCK loads issued together.
template <class T>
__device__ __forceinline__ T partition_prefix(const T* part, u32 b) {
    static_assert(GS_SCAN_PARTS % GS_BLOCK == 0, "partitions split evenly over the threads");
    constexpr int N = GS_SCAN_PARTS / GS_BLOCK;
    T v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const u32 i = threadIdx.x + j * GS_BLOCK;
        v[j] = part[i < GS_SCAN_PARTS ? i : 0];
    }
    T s = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) s += threadIdx.x + j * GS_BLOCK < b ? v[j] : (T)0;
    return s;
}

// p[i] for i < end, else 0 (end > 0).  The load is issued whatever i is (at a
// clamped index), so the loads of an unrolled loop stay in flight together;
// a conditional load would sit in a branch of its own that waits for it.
__device__ __forceinline__ u32 load_or_zero(const u32* p, u32 i, u32 end) {
    const u32 v = p[i < end ? i : end - 1];
    return i < end ? v : 0u;
}

// N values scan_in(in, gather, i0 + j * stride) (0 at or beyond end > 0), their
// loads issued together: the gather indices first, then the values
template <int N>
__device__ __forceinline__ void scan_in_n(const u32* in, const u32* gather, u32 i0, u32 stride,
                                          u32 end, u32 (&v)[N]) {
    u32 idx[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const u32 i = i0 + j * stride;
        idx[j] = i < end ? i : end - 1;
    }
    if (gather) {
#pragma unroll
        for (int j = 0; j < N; ++j) idx[j] = gather[idx[j]];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = in[idx[j]];
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = i0 + j * stride < end ? v[j] : 0u;
}

struct ScanStore {
    u32* out;
    u32* total;
    __device__ void item(u32 i, u32 v, u32 ex) const { (void)v; out[i] = ex; }
    __device__ void finish(u32 t) const { if (total) *total = t; }
};

template <class Epi>
__global__ void __launch_bounds__(GS_BLOCK) scan_down_kernel(const u32* in, const u32* gather,
                                                             const u32* n_dev, u32 n_host,
                                                             const u32* part, Epi epi) {
    __shared__ u32 lds4[4];
    u32 carry = partition_prefix(part, blockIdx.x);
    u32 before;
    block_exclusive_scan(carry, lds4, before);
    carry = before;
    u32 beg, end;
    chunk_of(dev_len(n_dev, n_host), GS_SCAN_PARTS, blockIdx.x, beg, end);
    for (u32 base = beg; base < end; base += GS_BLOCK * 4) {
        u32 v[4];
        u32 s = 0;
        const u32 i0 = base + threadIdx.x * 4;
        scan_in_n<4>(in, gather, i0, 1u, end, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) s += v[j];
        u32 total;
        u32 ex = block_exclusive_scan(s, lds4, total) + carry;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < end) epi.item(i0 + j, v[j], ex);
            ex += v[j];
        }
        carry += total;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) epi.finish(carry);
}

// ------------------------------------------------------------------------
// Launch helpers implemented in the .hip files
// ------------------------------------------------------------------------
// fill a u32 array with a value (graph-capture safe replacement for memset)
gs_status gs_fill_u32(u32* p, u32 value, int64_t count, hipStream_t s);

// exclusive scan of u32 values; the length is n_dev[0] when n_dev != NULL,
// else n_host.  total (device, may be NULL) receives the sum.  `part` needs
// GS_SCAN_PARTS + 1 u32.  gather (may be NULL): scan in[gather[i]] instead of
// in[i].  (A one-workgroup scan for short arrays was measured: 43 us for 62720
// values, latency-bound, against 12 us for the multi-workgroup scan.)
gs_status gs_scan_exclusive(const u32* in, u32* out, const u32* n_dev, u32 n_host, u32* total,
                            u32* part, hipStream_t s, const u32* gather = nullptr);
// the first launch of a scan: one partial sum per partition into part[0..GS_SCAN_PARTS)
gs_status gs_scan_reduce(const u32* in, const u32* gather, const u32* n_dev, u32 n_host, u32* part,
                         hipStream_t s);

// stable LSD radix sort on the low `bits` bits (8-bit digits; per pass a count
// kernel, an exclusive scan and a scatter kernel).  Buffers k[0]/v[0] hold the
// input; *slot receives the buffer index (0 or 1) that holds the result.  The
// length is n_dev[0] when n_dev != NULL, else n_host, and never exceeds
// `capacity` (< 2^30).  `scratch` needs gs_radix_scratch_bytes(capacity, bits).
// balanced: digits of equal width (ceil(bits / passes)) instead of 8 bits and a
// narrower last digit; the pass count, and so the result slot, is the same.
// unstable_first: the first pass may place equal digits in any order (cheaper
// ranking); the result is then ordered by key, but pairs with equal keys are
// not in input order, so only a caller that orders them itself afterwards
// may ask for it.
gs_status gs_radix_sort(u32* k[2], u32* v[2], const u32* n_dev, u32 n_host, int64_t capacity,
                        int bits, void* scratch, int* slot, hipStream_t s, bool balanced = false,
                        bool unstable_first = false);
uint64_t gs_radix_scratch_bytes(int64_t capacity, int bits);

// sigma3: bin by 3-sigma squares (GS_RASTER_FOOTPRINT_3SIGMA) instead of the
// opacity-aware ellipse; recorded in the frame for the binning that follows
gs_status gs_launch_project(gs_frame* f, const gs_gaussians* g, const gs_camera* cams,
                            float near_plane, bool sigma3, hipStream_t s);
// heavy_first: also build the heavy-first tile order (persistent launches);
// presort: order the visible entries by depth before emission instead of
// sorting each tile's list afterwards (GS_RASTER_DEPTH_PRESORT)
// balanced: balanced digit widths in the radix sort by tile (GS_RASTER_BALANCED_DIGITS)
gs_status gs_launch_bin(gs_frame* f, hipStream_t s, bool heavy_first, bool presort, bool balanced);
// targets (may be NULL): the L1 term of Eq. 3 fused in (gs_composite_l1)
gs_status gs_launch_raster_fwd(gs_frame* f, const gs_raster_opts* o, float* images,
                               const float* targets, float l1_scale, float* loss, float* dL,
                               hipStream_t s);
gs_status gs_launch_raster_bwd(gs_frame* f, const gs_raster_opts* o, const float* dL,
                               hipStream_t s);
// adam (may be NULL): the arrays it selects take their sparse Adam step
// instead of having their gradient written (gs_project_backward_adam)
gs_status gs_launch_project_bwd(gs_frame* f, const gs_gaussians* g, const gs_camera* cams,
                                float near_plane, const gs_gaussian_grads* gr, float* accum,
                                float* denom, bool rendered_only, const gs_fused_adam* adam,
                                hipStream_t s);

// ------------------------------------------------------------------------
// Device helpers
// ------------------------------------------------------------------------
#ifdef __HIPCC__
// One element of the sparse Adam step: the update when upd, else the values
// as read.  m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m c1) / (sqrt(v c2) + eps), c1, c2 the bias-correction factors.
// Shared by the optimiser kernel and the projection adjoint's fused step, so
// both give the same bits.
__device__ __forceinline__ void adam_element(bool upd, float g, float& m, float& v, float& p,
                                             float lr, float b1, float b2, float eps, float c1,
                                             float c2) {
    const float mn = fmaf(b1, m, (1.f - b1) * g);
    const float vn = fmaf(b2, v, (1.f - b2) * g * g);
    if (upd) {
        m = mn;
        v = vn;
        p -= lr * (mn * c1) / (sqrtf(vn * c2) + eps);
    }
}

// The bias-correction factors 1 / (1 - b^t) of step t, in FP64 rounded once.
__host__ __device__ __forceinline__ float adam_bias_factor(float b, int64_t t) {
    return (float)(1.0 / (1.0 - pow((double)b, (double)t)));
}

__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of `mask` in lanes below the calling lane
__device__ __forceinline__ u32 popc_below(u64 mask) {
    return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
}

// DPP move with a compile-time control word; lanes whose source is outside
// the row (or whose row is masked off) read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_mov_zero(float x) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROW_MASK, 0xF, true));
}

// Sum over the 64 lanes of a wave; the total lands in lane 63.  Must be
// called with all 64 lanes active.  row_shr 1/2/4/8 builds each row's
// inclusive prefix, row_bcast15 and row_bcast31 carry it across rows.
__device__ __forceinline__ float wave_sum_lane63(float x) {
    x += dpp_mov_zero<0x111, 0xF>(x);  // row_shr:1
    x += dpp_mov_zero<0x112, 0xF>(x);  // row_shr:2
    x += dpp_mov_zero<0x114, 0xF>(x);  // row_shr:4
    x += dpp_mov_zero<0x118, 0xF>(x);  // row_shr:8
    x += dpp_mov_zero<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_mov_zero<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// A projected splat is three float4: (mean hi x, y, mean lo x, y), (l11, l21,
// l22, opacity), (r, g, b, pad).  L = [l11 0; l21 l22] is the Cholesky factor
// of kappa Q, Q the conic (inverse screen-space covariance) and kappa =
// log2(e)/2, so G = exp(-d^T Q d / 2) = 2^-(u^2 + v^2) with u = l11 dx + l21 dy
// and v = l22 dy: a sum of squares, free of the cancellation that a dx^2 +
// 2 b dx dy + c dy^2 suffers for elongated splats, and two FMAs per pixel.
#define GS_KAPPA_D 0.72134752044448170
#define GS_KAPPA ((float)GS_KAPPA_D)

// One lane's 2x2 pixel quad relative to a splat: column offsets dx0, dx1 =
// dx0 + 1, row offsets dy0, dy1 = dy0 + 1, the exponent coordinate
// u = l11 dx + l21 dy of each pixel (the other three from the first by adding
// l11 and l21) and (l22 dy)^2 per row.  Pixel i of the quad is column i & 1,
// row i >> 1.
struct Quad {
    float dx[2], dy[2], u[4], vv[2];
};

__device__ __forceinline__ void quad_setup(float4 p0, float4 p1, float pxc0, float pyc0, Quad& q) {
    q.dx[0] = (pxc0 - p0.x) - p0.z;
    q.dx[1] = q.dx[0] + 1.f;
    q.dy[0] = (pyc0 - p0.y) - p0.w;
    q.dy[1] = q.dy[0] + 1.f;
    q.u[0] = fmaf(p1.x, q.dx[0], p1.y * q.dy[0]);
    q.u[1] = q.u[0] + p1.x;
    q.u[2] = q.u[0] + p1.y;
    q.u[3] = q.u[1] + p1.y;
    const float v0 = p1.z * q.dy[0], v1 = v0 + p1.z;
    q.vv[0] = v0 * v0;
    q.vv[1] = v1 * v1;
}

// G of pixel i of the quad; the forward and the adjoint both evaluate it
// through this function, so they see bit-identical values.
__device__ __forceinline__ float quad_G(const Quad& q, int i) {
    return __builtin_amdgcn_exp2f(-fmaf(q.u[i], q.u[i], q.vv[i >> 1]));
}

// Squared radius of a splat's footprint ellipse in (u, v) coordinates:
// o G >= 1/255  <=>  u^2 + v^2 <= log2(255 o), inflated like the footprint
// rectangle.  Negative when o < 1/255 (empty footprint).
__device__ __forceinline__ float footprint_r2(float o) {
    const float k = (float)GS_FOOTPRINT_INFLATE;
    return log2f(255.0f * o) * (k * k);
}

// Tile columns [c0, c1] of tile row ty whose 16x16 squares the footprint
// ellipse of a splat meets (before clamping to the footprint rectangle).  The
// ellipse cut by the row band 16 ty <= y <= 16 ty + 16 spans, in x, from its
// leftmost to its rightmost point inside the band: the boundary's extreme
// points clamped to the band.  Counting (projection) and enumeration (instance
// emission) both evaluate this from the same stored FP32 splat with the same
// code, so they agree bit for bit; the per-splat constants are computed once
// and a row costs two square roots.
struct FootprintRows {
    float l21, l22, r2, ry, ds, il11, mx, hy, ly;
};

__device__ __forceinline__ FootprintRows footprint_rows(float4 p0, float4 p1) {
    FootprintRows f;
    f.l21 = p1.y;
    f.l22 = p1.z;
    f.r2 = footprint_r2(p1.w);
    const float R = sqrtf(fmaxf(f.r2, 0.f));
    f.ry = R / f.l22;                                                  // dy half-extent
    f.ds = f.l21 * R / (f.l22 * sqrtf(fmaf(f.l21, f.l21, f.l22 * f.l22)));  // dy of the leftmost point
    f.il11 = 1.0f / p1.x;
    f.mx = p0.x + p0.z;
    f.hy = p0.y;
    f.ly = p0.w;
    return f;
}

// Columns [c0, c1] (of width w, 1 / w = iw) whose squares the ellipse meets
// inside the row band y0 <= y <= y0 + h; false if it misses the band.
__device__ __forceinline__ bool footprint_band(const FootprintRows& f, float y0, float h, float iw,
                                               int& c0, int& c1) {
    float dya = (y0 - f.hy) - f.ly;
    float dyb = dya + h;
    if (dya > f.ry || dyb < -f.ry) return false;
    dya = fmaxf(dya, -f.ry);
    dyb = fminf(dyb, f.ry);
    const float dl = fminf(fmaxf(f.ds, dya), dyb);
    const float dr = fminf(fmaxf(-f.ds, dya), dyb);
    const float vl = f.l22 * dl, vr = f.l22 * dr;
    const float xl = (-__builtin_amdgcn_sqrtf(fmaxf(fmaf(-vl, vl, f.r2), 0.f)) - f.l21 * dl) * f.il11;
    const float xr = (__builtin_amdgcn_sqrtf(fmaxf(fmaf(-vr, vr, f.r2), 0.f)) - f.l21 * dr) * f.il11;
    c0 = (int)ceilf((f.mx + xl) * iw) - 1;   // w c + w >= x_left
    c1 = (int)floorf((f.mx + xr) * iw);      // w c <= x_right
    return true;
}

__device__ __forceinline__ bool footprint_row(const FootprintRows& f, int ty, int& c0, int& c1) {
    return footprint_band(f, (float)(GS_TILE * ty), (float)GS_TILE, 1.0f / GS_TILE, c0, c1);
}

// The 8x8 quadrants of tile (tx, ty) that the footprint ellipse meets: bit
// (q & 1) + 2 (q >> 1) for the quadrant at (8 (q & 1), 8 (q >> 1)), from the
// row test at half resolution.  Every pixel whose alpha reaches 1/255 lies in
// a quadrant of the mask.
__device__ __forceinline__ u32 quadrant_mask(const FootprintRows& f, int tx, int ty) {
    u32 m = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int c0, c1;
        if (footprint_band(f, (float)(GS_TILE * ty + 8 * h), 8.0f, 0.125f, c0, c1)) {
            const int cl = 2 * tx;
            if (c0 <= cl && cl <= c1) m |= 1u << (2 * h);
            if (c0 <= cl + 1 && cl + 1 <= c1) m |= 2u << (2 * h);
        }
    }
    return m;
}

// Number of tiles of row ty inside the rectangle columns [x0, x1]; the first
// of them in *first.
__device__ __forceinline__ u32 footprint_row_count(const FootprintRows& f, int ty, int x0, int x1,
                                                   int* first) {
    int c0, c1;
    if (!footprint_row(f, ty, c0, c1)) return 0;
    c0 = c0 > x0 ? c0 : x0;
    c1 = c1 < x1 ? c1 : x1;
    *first = c0;
    return c1 >= c0 ? (u32)(c1 - c0 + 1) : 0u;
}
#endif
