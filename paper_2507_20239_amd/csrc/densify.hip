// Densification (the split / clone / prune step of the paper's Preliminary,
// scheduled by its global-to-local strategy) as stream compaction, plus the
// statistic that drives it, the adaptive opacity threshold (Methodology,
// Adaptive Opacity Pruning) and the L1 term of the loss (Eq. 3).
//
// All elementwise passes are HBM-bound: one thread per Gaussian, coalesced
// SoA reads, no atomics, fixed order (bit-reproducible results).
#include <mutex>

#include "gs_internal.h"

namespace {

constexpr int STATS_VIEWS_PER_LAUNCH = 64;

struct ViewScale {
    float sx[STATS_VIEWS_PER_LAUNCH];
    float sy[STATS_VIEWS_PER_LAUNCH];
};

__global__ void __launch_bounds__(GS_BLOCK) stats_kernel(const float* __restrict__ g,
                                                         const int32_t* __restrict__ vis,
                                                         int v0, int vc, int64_t n,
                                                         ViewScale sc, float* accum,
                                                         float* denom) {
    const int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (i >= n) return;
    float a = accum[i], d = denom[i];
    // eight views' loads in flight at once, then their sums in view order
    // (the same additions in the same order as one view at a time)
    int k = 0;
    for (; k + 8 <= vc; k += 8) {
        int vv[8];
        float gx[8], gy[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t v = v0 + k + j;
            vv[j] = vis[v * n + i];
            gx[j] = g[(2 * v) * n + i];
            gy[j] = g[(2 * v + 1) * n + i];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (!vv[j]) continue;
            const float x = gx[j] * sc.sx[k + j];
            const float y = gy[j] * sc.sy[k + j];
            const float nrm = sqrtf(fmaf(x, x, y * y));
            a = a + nrm;
            d = d + 1.0f;
        }
    }
    for (; k < vc; ++k) {
        const int64_t v = v0 + k;
        if (!vis[v * n + i]) continue;
        const float gx = g[(2 * v) * n + i] * sc.sx[k];
        const float gy = g[(2 * v + 1) * n + i] * sc.sy[k];
        // sqrtf is correctly rounded under the default HIP flags (the _rn
        // intrinsic is a bare v_sqrt_f32 on gfx950, up to 1 ulp off)
        const float nrm = sqrtf(fmaf(gx, gx, gy * gy));
        a = a + nrm;
        d = d + 1.0f;
    }
    accum[i] = a;
    denom[i] = d;
}

__global__ void __launch_bounds__(GS_BLOCK) select_kernel(
    const float* __restrict__ accum, const float* __restrict__ denom,
    const float* __restrict__ log_scales, const float* __restrict__ logits, int64_t n,
    float tau_g, float ls_thr, float logit_thr, int mode, uint8_t* split, uint8_t* clone,
    uint8_t* prune) {
    const int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (i >= n) return;
    const float dn = denom[i];
    const float avg = dn > 0.f ? __fdiv_rn(accum[i], dn) : 0.f;
    float mx = log_scales[i];
    const float l1 = log_scales[n + i], l2 = log_scales[2 * n + i];
    if (l1 > mx) mx = l1;
    if (l2 > mx) mx = l2;
    const bool hot = avg >= tau_g;
    const bool big = mx > ls_thr;
    // the operation a hot Gaussian takes under this mode
    const bool sp = mode == GS_DENSIFY_SPLIT_ONLY || (mode != GS_DENSIFY_CLONE_ONLY && big);
    split[i] = (uint8_t)(hot && sp);
    clone[i] = (uint8_t)(hot && !sp && mode != GS_DENSIFY_SPLIT_LARGE);
    prune[i] = (uint8_t)(logits[i] < logit_thr);
}

__global__ void plan_count_kernel(const uint8_t* split, const uint8_t* clone, const uint8_t* prune,
                                  int64_t n, u32* cnt) {
    const int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (i >= n) return;
    // the three mask loads issued together (no short-circuit chain of waits)
    const uint8_t p = prune[i], sp = split[i], cl = clone[i];
    cnt[i] = p ? 0u : ((sp | cl) ? 2u : 1u);
}

__global__ void plan_write_kernel(const uint8_t* split, const uint8_t* clone, const uint8_t* prune,
                                  const u32* offs, int64_t n, int32_t* src, uint8_t* kind,
                                  int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (i >= n) return;
    const uint8_t p = prune[i], sp = split[i], cl = clone[i];
    const int64_t o = offs[i];
    if (p) return;
    uint8_t k0 = GS_KIND_KEEP, k1 = GS_KIND_KEEP;
    int rows = 1;
    if (sp) {
        k0 = GS_KIND_SPLIT0;
        k1 = GS_KIND_SPLIT1;
        rows = 2;
    } else if (cl) {
        k1 = GS_KIND_CLONE;
        rows = 2;
    }
    if (o < cap) {
        src[o] = (int32_t)i;
        kind[o] = k0;
    }
    if (rows == 2 && o + 1 < cap) {
        src[o + 1] = (int32_t)i;
        kind[o + 1] = k1;
    }
}

__global__ void plan_total_kernel(const u32* total, int64_t* n_out) { *n_out = (int64_t)*total; }

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 S-box; the
// key advances by the two Weyl increments between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, u32 k0, u32 k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const u32 lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const u32 lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Three normals for split child `child` of `parent` (Box-Muller in FP64).
__device__ __forceinline__ void split_normals(u64 seed, u64 step, int64_t parent, int child,
                                              float z[3], uint4* words) {
    const uint4 ctr = make_uint4((u32)((u64)parent & 0xffffffffu), (u32)((u64)parent >> 32),
                                 (u32)child, (u32)step);
    const uint4 x = philox10(ctr, (u32)(seed & 0xffffffffu), (u32)(seed >> 32));
    if (words) *words = x;
    const double s24 = 1.0 / 16777216.0;
    const double u1 = (double)((x.x >> 8) + 1u) * s24, u2 = (double)(x.y >> 8) * s24;
    const double u3 = (double)((x.z >> 8) + 1u) * s24, u4 = (double)(x.w >> 8) * s24;
    const double r = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    const double two_pi = 6.283185307179586476925286766559;
    double sn, cs;
    sincos(two_pi * u2, &sn, &cs);
    z[0] = (float)(r * cs);
    z[1] = (float)(r * sn);
    z[2] = (float)(r2 * cos(two_pi * u4));
}

__global__ void split_normals_kernel(const int64_t* parents, const int32_t* children, int64_t m,
                                     u64 seed, u64 step, uint4* words, float* z) {
    const int64_t k = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (k >= m) return;
    float zz[3];
    uint4 w;
    split_normals(seed, step, parents[k], children[k], zz, &w);
    words[k] = w;
    z[3 * k] = zz[0];
    z[3 * k + 1] = zz[1];
    z[3 * k + 2] = zz[2];
}

// Every attribute of the compaction in one pass: a thread owns one output
// slot, reads its source index and kind once, and writes that slot of every
// row of every attribute (rows of one attribute four at a time, so their loads
// are in flight together).  Consecutive threads touch consecutive slots of a
// row: the writes are sequential and the reads nearly so (sources ascend).
constexpr int APPLY_MAX_ATTRS = 24;

struct ApplyTable {
    gs_attr a[APPLY_MAX_ATTRS];
    int count;
};

// position of a kept or cloned Gaussian, or of a split child: the parent's
// mean plus R(q) diag(s) z with z from the Philox stream
__device__ __forceinline__ void apply_mean(const float* __restrict__ in, float* __restrict__ out,
                                           int64_t i, int64_t j, uint8_t k, int64_t n_in,
                                           int64_t n_out, const float* __restrict__ ls,
                                           const float* __restrict__ quats, u64 seed, u64 step) {
    float m0 = in[i], m1 = in[n_in + i], m2 = in[2 * n_in + i];
    if (k == GS_KIND_SPLIT0 || k == GS_KIND_SPLIT1) {
        float z[3];
        split_normals(seed, step, i, k == GS_KIND_SPLIT1 ? 1 : 0, z, nullptr);
        const float v0 = expf(ls[i]) * z[0], v1 = expf(ls[n_in + i]) * z[1],
                    v2 = expf(ls[2 * n_in + i]) * z[2];
        float qw = quats[i], qx = quats[n_in + i], qy = quats[2 * n_in + i], qz = quats[3 * n_in + i];
        const float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        qw *= inv; qx *= inv; qy *= inv; qz *= inv;
        const float R00 = 1.f - 2.f * (qy * qy + qz * qz), R01 = 2.f * (qx * qy - qw * qz),
                    R02 = 2.f * (qx * qz + qw * qy);
        const float R10 = 2.f * (qx * qy + qw * qz), R11 = 1.f - 2.f * (qx * qx + qz * qz),
                    R12 = 2.f * (qy * qz - qw * qx);
        const float R20 = 2.f * (qx * qz - qw * qy), R21 = 2.f * (qy * qz + qw * qx),
                    R22 = 1.f - 2.f * (qx * qx + qy * qy);
        m0 += R00 * v0 + R01 * v1 + R02 * v2;
        m1 += R10 * v0 + R11 * v1 + R12 * v2;
        m2 += R20 * v0 + R21 * v1 + R22 * v2;
    }
    out[j] = m0;
    out[n_out + j] = m1;
    out[2 * n_out + j] = m2;
}

__global__ void __launch_bounds__(GS_BLOCK) apply_kernel(ApplyTable t, const int32_t* __restrict__ src,
                                                         const uint8_t* __restrict__ kind,
                                                         int64_t n_in, int64_t n_out,
                                                         const float* __restrict__ ls,
                                                         const float* __restrict__ quats, u64 seed,
                                                         u64 step) {
    const int64_t j = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (j >= n_out) return;
    const int64_t i = src[j];
    const uint8_t k = kind[j];
    const bool split = k == GS_KIND_SPLIT0 || k == GS_KIND_SPLIT1;
    // both rows of a cloned parent: its KEEP row is followed by its CLONE row
    const bool cloned = k == GS_KIND_CLONE ||
                        (k == GS_KIND_KEEP && j + 1 < n_out && kind[j + 1] == GS_KIND_CLONE);
    for (int a = 0; a < t.count; ++a) {
        const gs_attr at = t.a[a];
        const float* in = at.in;
        float* out = at.out;
        if (at.policy == GS_ATTR_MEAN) {
            apply_mean(in, out, i, j, k, n_in, n_out, ls, quats, seed, step);
            continue;
        }
        const bool zero = at.policy == GS_ATTR_ZERO || (at.policy == GS_ATTR_ZERO_NEW && k != GS_KIND_KEEP);
        // log-scales of split children shrink by 1.6 (ln 1.6 subtracted); a
        // lineage counter of the row's operation grows by one
        float sub = 0.f;
        if (at.policy == GS_ATTR_LOGSCALE && split) sub = 0.47000362924573558f;
        if ((at.policy == GS_ATTR_SPLIT_COUNT && split) || (at.policy == GS_ATTR_CLONE_COUNT && cloned))
            sub = -1.f;
        int r = 0;
        for (; r + 4 <= at.rows; r += 4) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = zero ? 0.f : in[(int64_t)(r + u) * n_in + i];
#pragma unroll
            for (int u = 0; u < 4; ++u) out[(int64_t)(r + u) * n_out + j] = zero ? 0.f : v[u] - sub;
        }
        for (; r < at.rows; ++r)
            out[(int64_t)r * n_out + j] = zero ? 0.f : in[(int64_t)r * n_in + i] - sub;
    }
}

// --- adaptive opacity threshold: radix select of the k-th smallest logit ---
__device__ __forceinline__ u32 float_order_key(float f) {
    const u32 b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float float_from_order_key(u32 k) {
    const u32 b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

// --- spatial order: Morton (Z-order) codes of the means --------------------
// box: order keys of min x, y, z (slots 0..2) and of max x, y, z (3..5) over
// the finite means, reduced with integer atomics on the order keys.
__global__ void box_init_kernel(u32* box) {
    const int t = threadIdx.x;
    if (t < 6) box[t] = t < 3 ? 0xffffffffu : 0u;
}

__global__ void __launch_bounds__(GS_BLOCK) box_kernel(const float* __restrict__ means, int64_t n,
                                                       u32* box) {
    u32 lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
    const int64_t stride = (int64_t)gridDim.x * GS_BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x; i < n; i += stride) {
        const float x = means[i], y = means[n + i], z = means[2 * n + i];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) continue;
        const u32 k[3] = {float_order_key(x), float_order_key(y), float_order_key(z)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = min(lo[a], k[a]);
            hi[a] = max(hi[a], k[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            lo[a] = min(lo[a], (u32)__shfl_xor((int)lo[a], off, 64));
            hi[a] = max(hi[a], (u32)__shfl_xor((int)hi[a], off, 64));
        }
    }
    // the workgroup's four waves through LDS, then one atomic per bound and
    // workgroup (the grid is a few hundred workgroups: six addresses take every
    // atomic, so their number is what costs)
    __shared__ u32 s_box[GS_BLOCK / 64][6];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            s_box[w][a] = lo[a];
            s_box[w][3 + a] = hi[a];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        u32 v = s_box[0][a];
        for (int j = 1; j < GS_BLOCK / 64; ++j) v = a < 3 ? min(v, s_box[j][a]) : max(v, s_box[j][a]);
        if (a < 3) atomicMin(&box[a], v);
        else atomicMax(&box[a], v);
    }
}

// the low 10 bits of q spread to every third bit
__device__ __forceinline__ u32 spread3(u32 q) {
    q &= 0x3ffu;
    q = (q | (q << 16)) & 0x030000ffu;
    q = (q | (q << 8)) & 0x0300f00fu;
    q = (q | (q << 4)) & 0x030c30c3u;
    q = (q | (q << 2)) & 0x09249249u;
    return q;
}

// code = interleaved bits of the cell (qx, qy, qz) of a 1024^3 grid over the
// bounding box's cube (side = its longest extent), qx in bit 0; a non-finite
// mean gets the largest code.  FP32: d = x - lo, q = min(1023, trunc(d * (1024 / side))).
__global__ void __launch_bounds__(GS_BLOCK) morton_kernel(const float* __restrict__ means, int64_t n,
                                                          const u32* box, u32* codes, u32* idx) {
    const int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (i >= n) return;
    float lo[3], side = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = float_from_order_key(box[a]);
        side = fmaxf(side, float_from_order_key(box[3 + a]) - lo[a]);
    }
    const float inv = side > 0.f ? 1024.0f / side : 0.f;
    const float p[3] = {means[i], means[n + i], means[2 * n + i]};
    u32 code = 0x3fffffffu;
    if (isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2])) {
        code = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float t = (p[a] - lo[a]) * inv;
            const u32 q = t >= 1023.0f ? 1023u : (u32)t;
            code |= spread3(q) << a;
        }
    }
    codes[i] = code;
    idx[i] = (u32)i;
}

__global__ void fill_u8_kernel(uint8_t* p, uint8_t v, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * GS_BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x; i < n; i += stride) p[i] = v;
}

// state: [0] prefix, [1] prefix mask, [2] remaining rank; hist: 256 counters
__global__ void select_init_kernel(u32* state, u32* hist, u32 k) {
    const int t = threadIdx.x;
    hist[t] = 0;
    if (t == 0) {
        state[0] = 0;
        state[1] = 0;
        state[2] = k;
    }
}

__global__ void __launch_bounds__(GS_BLOCK) select_hist_kernel(const float* __restrict__ x,
                                                               int64_t n, const u32* state,
                                                               int shift, u32* hist) {
    __shared__ u32 h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const u32 prefix = state[0], mask = state[1];
    const int64_t stride = (int64_t)gridDim.x * GS_BLOCK;
    for (int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x; i < n; i += stride) {
        const u32 key = float_order_key(x[i]);
        if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void __launch_bounds__(256) select_pick_kernel(u32* state, u32* hist, int shift) {
    __shared__ u32 c[256];
    const int t = threadIdx.x;
    c[t] = hist[t];
    __syncthreads();
    if (t == 0) {
        u32 k = state[2], acc = 0;
        int d = 0;
        for (; d < 255; ++d) {
            if (acc + c[d] > k) break;
            acc += c[d];
        }
        state[0] |= (u32)d << shift;
        state[1] |= 255u << shift;
        state[2] = k - acc;
    }
    __syncthreads();
    hist[t] = 0;
}

__global__ void select_finish_kernel(const u32* state, float upper, float* thr) {
    const float v = float_from_order_key(state[0]);
    *thr = v < upper ? v : upper;
}

// --- L1 loss ---
__global__ void __launch_bounds__(GS_BLOCK) l1_kernel(const float* __restrict__ img,
                                                      const float* __restrict__ tgt, int64_t n,
                                                      float scale, float* loss, float* grad) {
    __shared__ float red[GS_BLOCK / 64];
    float acc = 0.f;
    const int64_t stride = (int64_t)gridDim.x * GS_BLOCK;
    const int64_t tid = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    // 16-byte vector body when all three arrays are 16-byte aligned, scalar tail
    const bool vec = ((((uintptr_t)img) | ((uintptr_t)tgt) | ((uintptr_t)grad)) & 15) == 0;
    const int64_t n4 = vec ? n / 4 : 0;
    const float4* img4 = (const float4*)img;
    const float4* tgt4 = (const float4*)tgt;
    float4* grad4 = (float4*)grad;
    for (int64_t i = tid; i < n4; i += stride) {
        const float4 a = img4[i], b = tgt4[i];
        const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z, d3 = a.w - b.w;
        grad4[i] = make_float4(d0 > 0.f ? scale : (d0 < 0.f ? -scale : 0.f),
                               d1 > 0.f ? scale : (d1 < 0.f ? -scale : 0.f),
                               d2 > 0.f ? scale : (d2 < 0.f ? -scale : 0.f),
                               d3 > 0.f ? scale : (d3 < 0.f ? -scale : 0.f));
        acc += (fabsf(d0) + fabsf(d1)) + (fabsf(d2) + fabsf(d3));
    }
    for (int64_t i = 4 * n4 + tid; i < n; i += stride) {
        const float d = img[i] - tgt[i];
        grad[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
        acc += fabsf(d);
    }
    acc = wave_sum_lane63(acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 63) red[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int k = 0; k < GS_BLOCK / 64; ++k) s += red[k];
        unsafeAtomicAdd(loss, s * scale);
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + GS_BLOCK - 1) / GS_BLOCK); }

// The compaction map: per-parent row counts, their exclusive scan (in place)
// and the rows.  cnt holds n words, part GS_SCAN_PARTS + 2 (the last one
// receives the total).
gs_status plan_enqueue(const uint8_t* split, const uint8_t* clone, const uint8_t* prune, int64_t n,
                       int32_t* src, uint8_t* kind, int64_t capacity, int64_t* n_out, u32* cnt,
                       u32* part, hipStream_t s) {
    u32* total = part + GS_SCAN_PARTS + 1;
    if (n > 0) {
        plan_count_kernel<<<blocks_for(n), GS_BLOCK, 0, s>>>(split, clone, prune, n, cnt);
        GS_TRY(gs_check_launch("plan_count"));
        GS_TRY(gs_scan_exclusive(cnt, cnt, nullptr, (u32)n, total, part, s));
        plan_write_kernel<<<blocks_for(n), GS_BLOCK, 0, s>>>(split, clone, prune, cnt, n, src, kind,
                                                             capacity);
        GS_TRY(gs_check_launch("plan_write"));
    } else {
        GS_TRY(gs_fill_u32(total, 0u, 1, s));
    }
    plan_total_kernel<<<1, 1, 0, s>>>(total, n_out);
    return gs_check_launch("plan_total");
}

// ---- scratch of the allocation-free plan --------------------------------
// gs_densify_plan_noalloc keeps its scan scratch (row counts of up to
// NOALLOC_PLAN_MAX parents, then the scan's partition sums) in this
// file-scope device array instead of a caller workspace.  Each GPU holds its
// own copy until the process ends.  In host code the name `scratch` is a
// host-side stand-in, not a device address: the device address is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// only that address is handed to kernels.
constexpr int64_t NOALLOC_PLAN_MAX = (int64_t)1 << 23;
constexpr int64_t NOALLOC_PART_WORDS = GS_SCAN_PARTS + 64;
static __device__ __align__(256) u32 scratch[NOALLOC_PLAN_MAX + NOALLOC_PART_WORDS];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
u32* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};

gs_status scratch_of_current_device(u32** out) {
    int dev = 0;
    GS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return gs_fail(GS_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return gs_fail(GS_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                           hipGetErrorString(e));
        g_scratch_dev[dev] = (u32*)p;
    }
    *out = g_scratch_dev[dev];
    return GS_OK;
}

}  // namespace

extern "C" {

gs_status gs_accumulate_densify_stats(const float* dmean2d, const int32_t* visible,
                                      const int32_t* view_wh, int32_t n_views, int64_t n,
                                      float* accum, float* denom, void* stream) {
    if (n < 0 || n_views < 0) return gs_fail(GS_ERR_INVALID, "negative size");
    if (n == 0 || n_views == 0) return GS_OK;
    if (!dmean2d || !visible || !view_wh || !accum || !denom)
        return gs_fail(GS_ERR_INVALID, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    for (int v0 = 0; v0 < n_views; v0 += STATS_VIEWS_PER_LAUNCH) {
        const int vc = (n_views - v0) < STATS_VIEWS_PER_LAUNCH ? (n_views - v0) : STATS_VIEWS_PER_LAUNCH;
        ViewScale sc;
        for (int k = 0; k < STATS_VIEWS_PER_LAUNCH; ++k) {
            sc.sx[k] = k < vc ? (float)view_wh[2 * (v0 + k)] * 0.5f : 0.f;
            sc.sy[k] = k < vc ? (float)view_wh[2 * (v0 + k) + 1] * 0.5f : 0.f;
        }
        stats_kernel<<<blocks_for(n), GS_BLOCK, 0, s>>>(dmean2d, visible, v0, vc, n, sc, accum, denom);
        GS_TRY(gs_check_launch("stats"));
    }
    return GS_OK;
}

gs_status gs_densify_select(const float* accum, const float* denom, const float* log_scales,
                            const float* opacity_logits, int64_t n, float grad_threshold,
                            float log_scale_threshold, float logit_threshold, int32_t mode,
                            uint8_t* split, uint8_t* clone, uint8_t* prune, void* stream) {
    if (n < 0) return gs_fail(GS_ERR_INVALID, "negative size");
    if (mode < GS_DENSIFY_SPLIT_LARGE || mode > GS_DENSIFY_CLONE_ONLY)
        return gs_fail(GS_ERR_INVALID, "unknown densification mode %d", mode);
    if (n == 0) return GS_OK;
    if (!accum || !denom || !log_scales || !opacity_logits || !split || !clone || !prune)
        return gs_fail(GS_ERR_INVALID, "null pointer");
    select_kernel<<<blocks_for(n), GS_BLOCK, 0, (hipStream_t)stream>>>(
        accum, denom, log_scales, opacity_logits, n, grad_threshold, log_scale_threshold,
        logit_threshold, mode, split, clone, prune);
    return gs_check_launch("densify_select");
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

gs_status gs_densify_plan_workspace_size(int64_t n, uint64_t* bytes) {
    if (n < 0 || !bytes) return gs_fail(GS_ERR_INVALID, "bad argument");
    *bytes = align256(4 * (uint64_t)(n > 0 ? n : 1)) + align256(4 * (GS_SCAN_PARTS + 2));
    return GS_OK;
}

gs_status gs_densify_plan(const uint8_t* split, const uint8_t* clone, const uint8_t* prune,
                          int64_t n, int32_t* src, uint8_t* kind, int64_t capacity,
                          int64_t* n_out, void* workspace, uint64_t workspace_bytes,
                          void* stream) {
    if (n < 0 || n >= (int64_t)1 << 31 || capacity < 0)
        return gs_fail(GS_ERR_INVALID, "n must be in [0, 2^31)");
    if (!n_out || !workspace || (n > 0 && (!split || !clone || !prune)) || (capacity > 0 && (!src || !kind)))
        return gs_fail(GS_ERR_INVALID, "null pointer");
    uint64_t need;
    gs_densify_plan_workspace_size(n, &need);
    if (workspace_bytes < need) return gs_fail(GS_ERR_INVALID, "workspace too small (%llu < %llu)",
                                               (unsigned long long)workspace_bytes,
                                               (unsigned long long)need);
    u32* cnt = (u32*)workspace;
    u32* part = (u32*)((char*)workspace + align256(4 * (uint64_t)(n > 0 ? n : 1)));
    return plan_enqueue(split, clone, prune, n, src, kind, capacity, n_out, cnt, part,
                        (hipStream_t)stream);
}

gs_status gs_densify_plan_noalloc(const uint8_t* split, const uint8_t* clone,
                                  const uint8_t* prune, int64_t n, int32_t* src, uint8_t* kind,
                                  int64_t capacity, int64_t* n_out, void* stream) {
    if (n < 0 || capacity < 0) return gs_fail(GS_ERR_INVALID, "n and capacity must be >= 0");
    if (n > NOALLOC_PLAN_MAX)
        return gs_fail(GS_ERR_INVALID,
                       "gs_densify_plan_noalloc takes at most %lld parents (got %lld); use "
                       "gs_densify_plan with a workspace", (long long)NOALLOC_PLAN_MAX, (long long)n);
    if (!n_out || (n > 0 && (!split || !clone || !prune)) || (capacity > 0 && (!src || !kind)))
        return gs_fail(GS_ERR_INVALID, "null pointer");
    u32* sc = nullptr;
    GS_TRY(scratch_of_current_device(&sc));
    return plan_enqueue(split, clone, prune, n, src, kind, capacity, n_out, sc,
                        sc + NOALLOC_PLAN_MAX, (hipStream_t)stream);
}

gs_status gs_densify_apply(const int32_t* src, const uint8_t* kind, int64_t n_out, int64_t n_in,
                           const gs_attr* attrs, int32_t n_attrs, const float* parent_means,
                           const float* parent_log_scales, const float* parent_quats,
                           uint64_t seed, uint64_t step, void* stream) {
    if (n_out < 0 || n_in < 0 || n_attrs < 0 || n_attrs > APPLY_MAX_ATTRS)
        return gs_fail(GS_ERR_INVALID, "bad sizes");
    if (n_out == 0) return GS_OK;
    if (!src || !kind || (n_attrs > 0 && !attrs)) return gs_fail(GS_ERR_INVALID, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    for (int a = 0; a < n_attrs; ++a) {
        const gs_attr& at = attrs[a];
        if (!at.out || at.rows <= 0 || (at.policy != GS_ATTR_ZERO && !at.in))
            return gs_fail(GS_ERR_INVALID, "attribute %d: bad pointer or rows", a);
        if (at.policy < GS_ATTR_COPY || at.policy > GS_ATTR_CLONE_COUNT)
            return gs_fail(GS_ERR_INVALID, "attribute %d: unknown policy %d", a, at.policy);
        if (at.policy == GS_ATTR_MEAN) {
            if (at.rows != 3 || !parent_log_scales || !parent_quats)
                return gs_fail(GS_ERR_INVALID, "attribute %d: MEAN needs rows=3, scales and quats", a);
        }
    }
    (void)parent_means;
    if (n_attrs == 0) return GS_OK;
    ApplyTable t;
    t.count = n_attrs;
    for (int a = 0; a < n_attrs; ++a) t.a[a] = attrs[a];
    apply_kernel<<<blocks_for(n_out), GS_BLOCK, 0, s>>>(t, src, kind, n_in, n_out, parent_log_scales,
                                                        parent_quats, seed, step);
    return gs_check_launch("densify_apply");
}

gs_status gs_split_normals(const int64_t* parents, const int32_t* children, int64_t m,
                           uint64_t seed, uint64_t step, uint32_t* words, float* z, void* stream) {
    if (m < 0) return gs_fail(GS_ERR_INVALID, "negative size");
    if (m == 0) return GS_OK;
    if (!parents || !children || !words || !z) return gs_fail(GS_ERR_INVALID, "null pointer");
    split_normals_kernel<<<blocks_for(m), GS_BLOCK, 0, (hipStream_t)stream>>>(
        parents, children, m, seed, step, (uint4*)words, z);
    return gs_check_launch("split_normals");
}

gs_status gs_spatial_order_workspace_size(int64_t n, uint64_t* bytes) {
    if (n < 0 || n >= ((int64_t)1 << 30) || !bytes) return gs_fail(GS_ERR_INVALID, "bad argument");
    const uint64_t nb = align256(4 * (uint64_t)(n > 0 ? n : 1));
    *bytes = 3 * nb + align256(gs_radix_scratch_bytes(n, 30)) + 256;
    return GS_OK;
}

gs_status gs_spatial_order(const float* means, int64_t n, int32_t* src, uint8_t* kind,
                           void* workspace, uint64_t workspace_bytes, void* stream) {
    uint64_t need;
    GS_TRY(gs_spatial_order_workspace_size(n, &need));
    if (n == 0) return GS_OK;
    if (!means || !src || !kind || !workspace) return gs_fail(GS_ERR_INVALID, "null pointer");
    if (workspace_bytes < need) return gs_fail(GS_ERR_INVALID, "workspace too small (%llu < %llu)",
                                               (unsigned long long)workspace_bytes,
                                               (unsigned long long)need);
    hipStream_t s = (hipStream_t)stream;
    char* b = (char*)workspace;
    const uint64_t nb = align256(4 * (uint64_t)n);
    u32* k0 = (u32*)b;
    u32* k1 = (u32*)(b + nb);
    u32* v1 = (u32*)(b + 2 * nb);
    void* scratch = (void*)(b + 3 * nb);
    u32* box = (u32*)(b + 3 * nb + align256(gs_radix_scratch_bytes(n, 30)));
    box_init_kernel<<<1, 64, 0, s>>>(box);
    GS_TRY(gs_check_launch("spatial_box_init"));
    int64_t blocks = blocks_for(n);
    box_kernel<<<(unsigned)(blocks > 512 ? 512 : blocks), GS_BLOCK, 0, s>>>(means, n, box);
    GS_TRY(gs_check_launch("spatial_box"));
    morton_kernel<<<blocks_for(n), GS_BLOCK, 0, s>>>(means, n, box, k0, (u32*)src);
    GS_TRY(gs_check_launch("morton_codes"));
    // stable: equal codes keep index order; four passes end in slot 0 (src)
    u32* k[2] = {k0, k1};
    u32* v[2] = {(u32*)src, v1};
    int slot = 0;
    GS_TRY(gs_radix_sort(k, v, nullptr, (u32)n, n, 30, scratch, &slot, s));
    if (slot != 0) return gs_fail(GS_ERR_HIP, "spatial order ended in the wrong buffer");
    fill_u8_kernel<<<(unsigned)(blocks > 2048 ? 2048 : blocks), GS_BLOCK, 0, s>>>(kind, GS_KIND_KEEP, n);
    return gs_check_launch("spatial_kind");
}

gs_status gs_radix_select_workspace_size(int64_t n, uint64_t* bytes) {
    if (n < 0 || !bytes) return gs_fail(GS_ERR_INVALID, "bad argument");
    *bytes = 256 * 4 + 256;
    return GS_OK;
}

gs_status gs_adaptive_prune_threshold(const float* opacity_logits, int64_t n, int64_t k,
                                      float upper_logit, float* thr, void* workspace,
                                      uint64_t workspace_bytes, void* stream) {
    if (n <= 0 || n >= (int64_t)1 << 32) return gs_fail(GS_ERR_INVALID, "n must be in [1, 2^32)");
    if (k < 0 || k >= n) return gs_fail(GS_ERR_INVALID, "k must be in [0, n)");
    if (!opacity_logits || !thr || !workspace) return gs_fail(GS_ERR_INVALID, "null pointer");
    if (workspace_bytes < 256 * 4 + 256) return gs_fail(GS_ERR_INVALID, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    u32* hist = (u32*)workspace;
    u32* state = hist + 256;
    select_init_kernel<<<1, 256, 0, s>>>(state, hist, (u32)k);
    GS_TRY(gs_check_launch("select_init"));
    int64_t blocks = blocks_for(n);
    if (blocks > 2048) blocks = 2048;
    for (int shift = 24; shift >= 0; shift -= 8) {
        select_hist_kernel<<<(unsigned)blocks, GS_BLOCK, 0, s>>>(opacity_logits, n, state, shift, hist);
        select_pick_kernel<<<1, 256, 0, s>>>(state, hist, shift);
        GS_TRY(gs_check_launch("radix_select"));
    }
    select_finish_kernel<<<1, 1, 0, s>>>(state, upper_logit, thr);
    return gs_check_launch("select_finish");
}

gs_status gs_l1_loss_grad(const float* image, const float* target, int64_t numel, float scale,
                          float* loss, float* dL_dimage, void* stream) {
    if (numel < 0) return gs_fail(GS_ERR_INVALID, "negative size");
    if (numel == 0) return GS_OK;
    if (!image || !target || !loss || !dL_dimage) return gs_fail(GS_ERR_INVALID, "null pointer");
    int64_t blocks = blocks_for((numel + 3) / 4);
    if (blocks > 512) blocks = 512;
    l1_kernel<<<(unsigned)blocks, GS_BLOCK, 0, (hipStream_t)stream>>>(image, target, numel, scale,
                                                                      loss, dL_dimage);
    return gs_check_launch("l1_loss");
}

}  // extern "C"
