// Photometric loss of Eq. 3 and its gradient w.r.t. the rendered image:
//   L = (1 - lambda) mean |I - T| + lambda (1 - mean SSIM(I, T)),
// SSIM with the 3DGS window: an 11 x 11 Gaussian of standard deviation 1.5,
// zero padding, C1 = 0.01^2, C2 = 0.03^2, the mean over every channel and
// pixel.  With mu = G*I, nu = G*T, Exx = G*I^2, Eyy = G*T^2, Exy = G*(I T),
//   S = (2 mu nu + C1)(2 (Exy - mu nu) + C2) / ((mu^2 + nu^2 + C1)((Exx - mu^2) + (Eyy - nu^2) + C2)),
// and dL/dI(q) = -lambda/N [ (G*a)(q) + 2 I(q) (G*b)(q) + T(q) (G*c)(q) ] + (1-lambda)/N sign(I-T)(q)
// where a = dS/dmu, b = dS/dExx, c = dS/dExy are maps over the pixels p
// (G is symmetric, so correlating with it is convolving with it).
//
// Three launches per image: the forward computes S and (a, b, c) for a 32x16
// tile per workgroup from a 42x26 LDS patch (separable: a horizontal pass to
// 26x32 partial sums, then a vertical one, two output pixels per thread); the
// backward filters (a, b, c) the same way and combines them with I and T at
// each pixel; a one-workgroup launch sums the per-tile losses in a fixed
// order.  HBM-bound: about 44 B per channel-pixel over the two launches.
#include "gs_internal.h"

namespace {

constexpr int TW = 32;              // output tile width
constexpr int TH = 16;              // output tile height
constexpr int SR = 5;               // window radius
constexpr int PW = TW + 2 * SR;     // patch width (42)
constexpr int PH = TH + 2 * SR;     // patch height (26)
constexpr int OUT_PER_THREAD = TW * TH / 256;   // 2 output pixels per thread

struct Window {
    float g[2 * SR + 1];
};

__device__ __forceinline__ float rcp_refined(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, r, 1.f), r, r);
}

constexpr int PATCH = PH * PW;
constexpr int PATCH_STEPS = (PATCH + 255) / 256;   // patch elements per thread (5)

// Element k of this thread's share of the patch at (y0, x0): where it sits in
// the patch (r, q) and its offset in a plane, clamped into the image (so the
// load is always issued; `in` says whether the value is used or taken as 0).
struct PatchSlot {
    int r, q;
    int64_t o;
    bool in, valid;
};

__device__ __forceinline__ PatchSlot patch_slot(int t, int k, int H, int W, int y0, int x0) {
    PatchSlot p;
    const int i0 = t + 256 * k;
    p.valid = i0 < PATCH;
    const int i = p.valid ? i0 : PATCH - 1;
    p.r = i / PW;
    p.q = i % PW;
    const int y = y0 + p.r, x = x0 + p.q;
    p.in = y >= 0 && y < H && x >= 0 && x < W;
    p.o = (int64_t)min(max(y, 0), H - 1) * W + min(max(x, 0), W - 1);
    return p;
}

__global__ void __launch_bounds__(256) ssim_fwd_kernel(const float* __restrict__ img,
                                                       const float* __restrict__ tgt, int H, int W,
                                                       Window win, float lambda, float inv_n,
                                                       float* abc, float* partial) {
    __shared__ float sx[PH][PW], sy[PH][PW];
    __shared__ float h[5][PH][TW];
    __shared__ float red[2][4];
    const int c = blockIdx.z;
    const int64_t plane = (int64_t)H * W;
    const float* X = img + c * plane;
    const float* Y = tgt + c * plane;
    const int x0 = blockIdx.x * TW - SR, y0 = blockIdx.y * TH - SR;
    const int t = threadIdx.x;
    {
        // every patch load of the thread in flight before any is stored (zero
        // padding outside the image)
        float vx[PATCH_STEPS], vy[PATCH_STEPS];
#pragma unroll
        for (int k = 0; k < PATCH_STEPS; ++k) {
            const PatchSlot p = patch_slot(t, k, H, W, y0, x0);
            const float a = X[p.o], b = Y[p.o];
            vx[k] = p.in ? a : 0.f;
            vy[k] = p.in ? b : 0.f;
        }
#pragma unroll
        for (int k = 0; k < PATCH_STEPS; ++k) {
            const PatchSlot p = patch_slot(t, k, H, W, y0, x0);
            if (p.valid) {
                sx[p.r][p.q] = vx[k];
                sy[p.r][p.q] = vy[k];
            }
        }
    }
    __syncthreads();
    for (int i = t; i < PH * TW; i += 256) {
        const int r = i / TW, q = i % TW;
        float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
        for (int k = 0; k <= 2 * SR; ++k) {
            const float a = sx[r][q + k], b = sy[r][q + k], w = win.g[k];
            m0 = fmaf(w, a, m0);
            m1 = fmaf(w, b, m1);
            m2 = fmaf(w, a * a, m2);
            m3 = fmaf(w, b * b, m3);
            m4 = fmaf(w, a * b, m4);
        }
        h[0][r][q] = m0;
        h[1][r][q] = m1;
        h[2][r][q] = m2;
        h[3][r][q] = m3;
        h[4][r][q] = m4;
    }
    __syncthreads();
    const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
    const int64_t map = (int64_t)gridDim.z * plane;   // maps a, b, c one after the other
    float s_sum = 0.f, l1_sum = 0.f;
#pragma unroll
    for (int j = 0; j < OUT_PER_THREAD; ++j) {
        const int r = t / TW + j * (256 / TW), q = t % TW;
        float mu = 0.f, nu = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
        for (int k = 0; k <= 2 * SR; ++k) {
            const float w = win.g[k];
            mu = fmaf(w, h[0][r + k][q], mu);
            nu = fmaf(w, h[1][r + k][q], nu);
            exx = fmaf(w, h[2][r + k][q], exx);
            eyy = fmaf(w, h[3][r + k][q], eyy);
            exy = fmaf(w, h[4][r + k][q], exy);
        }
        const float A = fmaf(2.f * mu, nu, C1);
        const float B = fmaf(2.f, exy - mu * nu, C2);
        const float Cc = fmaf(mu, mu, fmaf(nu, nu, C1));
        const float D = (exx - mu * mu) + (eyy - nu * nu) + C2;
        // the four reciprocals once (hardware reciprocal + one Newton step)
        // instead of seven divisions
        const float rA = rcp_refined(A), rB = rcp_refined(B), rC = rcp_refined(Cc),
                    rD = rcp_refined(D);
        const float S = (A * B) * (rC * rD);
        const int py = blockIdx.y * TH + r, px = blockIdx.x * TW + q;
        if (py < H && px < W) {
            const int64_t o = c * plane + (int64_t)py * W + px;
            // dS/dmu, dS/dExx, dS/dExy
            abc[o] = S * fmaf(2.f * nu, rA - rB, 2.f * mu * (rD - rC));
            abc[map + o] = -S * rD;
            abc[2 * map + o] = 2.f * S * rB;
            s_sum += S;
            l1_sum += fabsf(sx[r + SR][q + SR] - sy[r + SR][q + SR]);
        }
    }
    // loss += inv_n ((1 - lambda) sum |I - T| + lambda sum (1 - S)) over this tile
    s_sum = wave_sum_lane63(s_sum);
    l1_sum = wave_sum_lane63(l1_sum);
    const int lane = t & 63, w = t >> 6;
    if (lane == 63) {
        red[0][w] = s_sum;
        red[1][w] = l1_sum;
    }
    __syncthreads();
    if (t == 0) {
        const float ssum = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        const float lsum = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        const int nin = (min(TH, H - (int)blockIdx.y * TH)) * (min(TW, W - (int)blockIdx.x * TW));
        const u32 b = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        partial[b] = inv_n * ((1.f - lambda) * lsum + lambda * ((float)nin - ssum));
    }
}

// loss[0] += the sum of the per-tile partial losses, in a fixed order (one
// workgroup; thousands of same-address atomics would serialise).
__global__ void __launch_bounds__(1024) loss_sum_kernel(const float* __restrict__ partial, u32 count,
                                                       float* loss) {
    __shared__ float red[16];
    float s = 0.f;
    for (u32 i = threadIdx.x; i < count; i += 1024) s += partial[i];
    s = wave_sum_lane63(s);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < 16; ++w) t += red[w];
        loss[0] += t;
    }
}

__global__ void __launch_bounds__(256) ssim_bwd_kernel(const float* __restrict__ img,
                                                       const float* __restrict__ tgt, int H, int W,
                                                       Window win, float lambda, float inv_n,
                                                       const float* __restrict__ abc,
                                                       float* __restrict__ grad) {
    __shared__ float sa[3][PH][PW];
    __shared__ float h[3][PH][TW];
    const int c = blockIdx.z;
    const int64_t plane = (int64_t)H * W;
    const int x0 = blockIdx.x * TW - SR, y0 = blockIdx.y * TH - SR;
    const int t = threadIdx.x;
    {
        float v[3][PATCH_STEPS];
#pragma unroll
        for (int k = 0; k < PATCH_STEPS; ++k) {
            const PatchSlot p = patch_slot(t, k, H, W, y0, x0);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const float a = abc[((int64_t)m * gridDim.z + c) * plane + p.o];
                v[m][k] = p.in ? a : 0.f;
            }
        }
#pragma unroll
        for (int k = 0; k < PATCH_STEPS; ++k) {
            const PatchSlot p = patch_slot(t, k, H, W, y0, x0);
            if (p.valid) {
#pragma unroll
                for (int m = 0; m < 3; ++m) sa[m][p.r][p.q] = v[m][k];
            }
        }
    }
    __syncthreads();
    for (int i = t; i < PH * TW; i += 256) {
        const int r = i / TW, q = i % TW;
        float m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
        for (int k = 0; k <= 2 * SR; ++k) {
            const float w = win.g[k];
            m0 = fmaf(w, sa[0][r][q + k], m0);
            m1 = fmaf(w, sa[1][r][q + k], m1);
            m2 = fmaf(w, sa[2][r][q + k], m2);
        }
        h[0][r][q] = m0;
        h[1][r][q] = m1;
        h[2][r][q] = m2;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < OUT_PER_THREAD; ++j) {
        const int r = t / TW + j * (256 / TW), q = t % TW;
        const int py = blockIdx.y * TH + r, px = blockIdx.x * TW + q;
        if (py >= H || px >= W) continue;
        float ga = 0.f, gb = 0.f, gc = 0.f;
#pragma unroll
        for (int k = 0; k <= 2 * SR; ++k) {
            const float w = win.g[k];
            ga = fmaf(w, h[0][r + k][q], ga);
            gb = fmaf(w, h[1][r + k][q], gb);
            gc = fmaf(w, h[2][r + k][q], gc);
        }
        const int64_t o = c * plane + (int64_t)py * W + px;
        const float I = img[o], Tt = tgt[o];
        const float dssim = fmaf(2.f * I, gb, ga) + Tt * gc;
        const float sgn = I > Tt ? 1.f : (I < Tt ? -1.f : 0.f);
        grad[o] = inv_n * ((1.f - lambda) * sgn - lambda * dssim);
    }
}

}  // namespace

extern "C" gs_status gs_ssim_workspace_size(int32_t channels, int32_t height, int32_t width,
                                            uint64_t* bytes) {
    if (channels <= 0 || height <= 0 || width <= 0 || !bytes)
        return gs_fail(GS_ERR_INVALID, "bad image size");
    // the maps a, b, c and one partial loss per 32 x 16 tile and channel
    const uint64_t tiles = (uint64_t)((width + TW - 1) / TW) * (uint64_t)((height + TH - 1) / TH);
    *bytes = 3ull * 4ull * (uint64_t)channels * (uint64_t)height * (uint64_t)width +
             4ull * tiles * (uint64_t)channels;
    return GS_OK;
}

extern "C" gs_status gs_ssim_loss_grad(const float* image, const float* target, int32_t channels,
                                       int32_t height, int32_t width, float lambda, float* loss,
                                       float* dL_dimage, void* workspace, uint64_t workspace_bytes,
                                       void* stream) {
    uint64_t need = 0;
    GS_TRY(gs_ssim_workspace_size(channels, height, width, &need));
    if (height > 16384 || width > 16384 || channels > 64)
        return gs_fail(GS_ERR_INVALID, "image larger than 64 x 16384 x 16384");
    if (!(lambda >= 0.f && lambda <= 1.f)) return gs_fail(GS_ERR_INVALID, "lambda must be in [0, 1]");
    if (!image || !target || !loss || !dL_dimage || !workspace)
        return gs_fail(GS_ERR_INVALID, "null pointer");
    if (workspace_bytes < need) return gs_fail(GS_ERR_INVALID, "workspace too small");
    Window win;
    double sum = 0.0, g[2 * SR + 1];
    for (int k = 0; k <= 2 * SR; ++k) {
        g[k] = exp(-(double)((k - SR) * (k - SR)) / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k <= 2 * SR; ++k) win.g[k] = (float)(g[k] / sum);
    const float inv_n = (float)(1.0 / ((double)channels * height * width));
    dim3 grid((unsigned)((width + TW - 1) / TW), (unsigned)((height + TH - 1) / TH), (unsigned)channels);
    hipStream_t s = (hipStream_t)stream;
    float* abc = (float*)workspace;
    float* partial = abc + 3ull * (uint64_t)channels * (uint64_t)height * (uint64_t)width;
    ssim_fwd_kernel<<<grid, 256, 0, s>>>(image, target, height, width, win, lambda, inv_n, abc,
                                         partial);
    GS_TRY(gs_check_launch("ssim_fwd"));
    loss_sum_kernel<<<1, 1024, 0, s>>>(partial, grid.x * grid.y * grid.z, loss);
    GS_TRY(gs_check_launch("loss_sum"));
    ssim_bwd_kernel<<<grid, 256, 0, s>>>(image, target, height, width, win, lambda, inv_n, abc,
                                         dL_dimage);
    return gs_check_launch("ssim_bwd");
}
