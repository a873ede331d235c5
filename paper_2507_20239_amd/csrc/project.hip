// Projection of 3D Gaussians into one or more views, and its adjoint.
//
// Forward (Preliminary of the paper: Sigma = R S S^T R^T, Sigma' = J W Sigma
// W^T J^T; Eq. 2's colour c_i from spherical harmonics): one thread per
// Gaussian, looping over the views so the parameters are read from HBM once
// (structure-of-arrays, coalesced).  The camera-space position and the
// screen-space mean are evaluated in FP64 (cheap on CDNA4 for this
// HBM-bound kernel) and the mean is stored as an FP32 hi/lo pair, which keeps
// the pixel offset exact to ~1e-7 px on 1600-pixel images.  The depth used
// for ordering is the FP32 rounding of the FP64 depth evaluated as a fused
// multiply-add chain.  Each (view, Gaussian) entry also gets its footprint:
// the tiles whose squares meet the ellipse o G >= 1/255, counted row by row,
// or with the 3-sigma option every tile of the square of half-side
// ceil(3 sqrt(largest eigenvalue of Sigma')).
//
// Adjoint: one thread per Gaussian again; it recomputes the projection
// (instead of storing intermediates), applies the chain rule to the raw
// parameters, sums over views in registers (deterministic, no atomics) and
// accumulates the densification statistic: the norm of the position
// gradient in NDC units (Preliminary, last paragraph), one term per view in
// which the Gaussian was rendered.
#include "gs_internal.h"

namespace {

// Real spherical-harmonic constants, Condon-Shortley phase:
// Y00 = 1/(2 sqrt(pi)); C1 = sqrt(3/(4 pi)); C2a = sqrt(15/(4 pi)); C2b = sqrt(5/(16 pi));
// C2c = sqrt(15/(16 pi)); C3a = sqrt(35/(32 pi)); C3b = sqrt(105/(4 pi));
// C3c = sqrt(21/(32 pi)); C3d = sqrt(7/(16 pi)); C3e = sqrt(105/(16 pi)).
constexpr float SH_Y00 = 0.28209479177387814f;
constexpr float SH_C1 = 0.4886025119029199f;
constexpr float SH_C2a = 1.0925484305920792f;
constexpr float SH_C2b = 0.31539156525252005f;
constexpr float SH_C2c = 0.5462742152960396f;
constexpr float SH_C3a = 0.5900435899266435f;
constexpr float SH_C3b = 2.890611442640554f;
constexpr float SH_C3c = 0.4570457994644658f;
constexpr float SH_C3d = 0.3731763325901154f;
constexpr float SH_C3e = 1.445305721320277f;

// The basis is evaluated in FP64 and rounded once to FP32: the higher
// degrees are differences of products of the direction's coordinates (x^2 -
// 3 y^2 and the like), which near their zeros would leave FP32 rounding far
// above the value, and the colour coefficients' gradient is the basis itself.
template <int DEG>
__device__ __forceinline__ void sh_eval(double x, double y, double z, float* Y) {
    Y[0] = SH_Y00;
    if (DEG >= 1) {
        Y[1] = (float)(-(double)SH_C1 * y);
        Y[2] = (float)((double)SH_C1 * z);
        Y[3] = (float)(-(double)SH_C1 * x);
    }
    if (DEG >= 2) {
        const double xx = x * x, yy = y * y, zz = z * z;
        Y[4] = (float)((double)SH_C2a * x * y);
        Y[5] = (float)(-(double)SH_C2a * y * z);
        Y[6] = (float)((double)SH_C2b * (2.0 * zz - xx - yy));
        Y[7] = (float)(-(double)SH_C2a * x * z);
        Y[8] = (float)((double)SH_C2c * (xx - yy));
        if (DEG >= 3) {
            Y[9] = (float)(-(double)SH_C3a * y * (3.0 * xx - yy));
            Y[10] = (float)((double)SH_C3b * x * y * z);
            Y[11] = (float)(-(double)SH_C3c * y * (4.0 * zz - xx - yy));
            Y[12] = (float)((double)SH_C3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
            Y[13] = (float)(-(double)SH_C3c * x * (4.0 * zz - xx - yy));
            Y[14] = (float)((double)SH_C3e * z * (xx - yy));
            Y[15] = (float)(-(double)SH_C3a * x * (xx - 3.0 * yy));
        }
    }
}

// The unit direction from the camera centre C = -R^T t to the mean (FP64) and
// the colour basis there; also the direction and 1/distance in FP32 for the
// adjoint of the direction.
template <int DEG>
__device__ __forceinline__ void view_basis(const gs_camera& c, const float mu[3], float* Y,
                                           float dir[3], float& idist) {
    const double cx = -((double)c.R[0] * c.t[0] + (double)c.R[3] * c.t[1] + (double)c.R[6] * c.t[2]);
    const double cy = -((double)c.R[1] * c.t[0] + (double)c.R[4] * c.t[1] + (double)c.R[7] * c.t[2]);
    const double cz = -((double)c.R[2] * c.t[0] + (double)c.R[5] * c.t[1] + (double)c.R[8] * c.t[2]);
    double dx = mu[0] - cx, dy = mu[1] - cy, dz = mu[2] - cz;
    const double id = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    dx *= id;
    dy *= id;
    dz *= id;
    sh_eval<DEG>(dx, dy, dz, Y);
    dir[0] = (float)dx;
    dir[1] = (float)dy;
    dir[2] = (float)dz;
    idist = (float)id;
}

// Gradient of each polynomial Y_k w.r.t. (x, y, z), contracted with w_k:
// out = sum_k w_k grad Y_k.
template <int DEG>
__device__ __forceinline__ void sh_grad_contract(float x, float y, float z, const float* w,
                                                 float& gx, float& gy, float& gz) {
    gx = gy = gz = 0.f;
    if (DEG >= 1) {
        gy -= SH_C1 * w[1];
        gz += SH_C1 * w[2];
        gx -= SH_C1 * w[3];
    }
    if (DEG >= 2) {
        gx += SH_C2a * y * w[4];
        gy += SH_C2a * x * w[4];
        gy -= SH_C2a * z * w[5];
        gz -= SH_C2a * y * w[5];
        gx -= 2.f * SH_C2b * x * w[6];
        gy -= 2.f * SH_C2b * y * w[6];
        gz += 4.f * SH_C2b * z * w[6];
        gx -= SH_C2a * z * w[7];
        gz -= SH_C2a * x * w[7];
        gx += 2.f * SH_C2c * x * w[8];
        gy -= 2.f * SH_C2c * y * w[8];
        if (DEG >= 3) {
            const float xx = x * x, yy = y * y, zz = z * z;
            gx -= SH_C3a * 6.f * x * y * w[9];
            gy -= SH_C3a * 3.f * (xx - yy) * w[9];
            gx += SH_C3b * y * z * w[10];
            gy += SH_C3b * x * z * w[10];
            gz += SH_C3b * x * y * w[10];
            gx += 2.f * SH_C3c * x * y * w[11];
            gy -= SH_C3c * (4.f * zz - xx - 3.f * yy) * w[11];
            gz -= 8.f * SH_C3c * y * z * w[11];
            gx -= 6.f * SH_C3d * x * z * w[12];
            gy -= 6.f * SH_C3d * y * z * w[12];
            gz += SH_C3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
            gx -= SH_C3c * (4.f * zz - 3.f * xx - yy) * w[13];
            gy += 2.f * SH_C3c * x * y * w[13];
            gz -= 8.f * SH_C3c * x * z * w[13];
            gx += 2.f * SH_C3e * x * z * w[14];
            gy -= 2.f * SH_C3e * y * z * w[14];
            gz += SH_C3e * (xx - yy) * w[14];
            gx -= SH_C3a * 3.f * (xx - yy) * w[15];
            gy += SH_C3a * 6.f * x * y * w[15];
        }
    }
}

struct ProjArgs {
    const float* means;
    const float* log_scales;
    const float* quats;
    const float* logits;
    const float* sh;
    int64_t n;
    int V;
    float near_plane;
    const gs_camera* cams;
    const gs_view_info* views;
    u32* depth_key;
    u32* tiles_touched;
    uint2* rect;
    float4* splat;
    float* splat_grad;     // [E][9], cleared here for the adjoint of this step
};

// Per-Gaussian activated parameters.
struct Activated {
    float s[3];        // scales
    float q[4];        // unit quaternion (w, x, y, z)
    float qnorm;
    float o;           // opacity
    float R[9];        // rotation, row-major
    float Sig[6];      // Sigma: 00 01 02 11 12 22
    double SigD[6];    // the same in FP64 (input of the screen-space covariance)
};

// Raw parameters of one Gaussian (structure-of-arrays loads).
struct Raw {
    float mu[3], ls[3], q[4], logit;
};

__device__ __forceinline__ Raw load_raw(const ProjArgs& a, int64_t i) {
    const int64_t n = a.n;
    Raw r;
#pragma unroll
    for (int k = 0; k < 3; ++k) r.mu[k] = a.means[k * n + i];
#pragma unroll
    for (int k = 0; k < 3; ++k) r.ls[k] = a.log_scales[k * n + i];
#pragma unroll
    for (int k = 0; k < 4; ++k) r.q[k] = a.quats[k * n + i];
    r.logit = a.logits[i];
    return r;
}

// Position, scales and opacity: all the culling test needs.
__device__ __forceinline__ void activate_light(const Raw& r, float mu[3], Activated& g) {
#pragma unroll
    for (int k = 0; k < 3; ++k) mu[k] = r.mu[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) g.s[k] = expf(r.ls[k]);
    g.o = 1.0f / (1.0f + expf(-r.logit));
}

// Rotation and covariance (Eq. 1: Sigma = R S S^T R^T).  Evaluated in FP64:
// an elongated Gaussian seen edge-on has a screen-space covariance whose
// determinant cancels to a few 1e-4 of its terms, so FP32 products here would
// leave the conic with relative errors far above FP32 rounding.
__device__ __forceinline__ void activate_rot(const Raw& r, Activated& g) {
    const double q0 = r.q[0], q1 = r.q[1], q2 = r.q[2], q3 = r.q[3];
    const double qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    g.qnorm = (float)qn;
    const double inv = 1.0 / qn;
    const double w = q0 * inv, x = q1 * inv, y = q2 * inv, z = q3 * inv;
    g.q[0] = (float)w; g.q[1] = (float)x; g.q[2] = (float)y; g.q[3] = (float)z;
    double R[9];
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
#pragma unroll
    for (int k = 0; k < 9; ++k) g.R[k] = (float)R[k];
    const double s0 = (double)g.s[0] * g.s[0], s1 = (double)g.s[1] * g.s[1],
                 s2 = (double)g.s[2] * g.s[2];
    double* S = g.SigD;
    S[0] = R[0] * R[0] * s0 + R[1] * R[1] * s1 + R[2] * R[2] * s2;
    S[1] = R[0] * R[3] * s0 + R[1] * R[4] * s1 + R[2] * R[5] * s2;
    S[2] = R[0] * R[6] * s0 + R[1] * R[7] * s1 + R[2] * R[8] * s2;
    S[3] = R[3] * R[3] * s0 + R[4] * R[4] * s1 + R[5] * R[5] * s2;
    S[4] = R[3] * R[6] * s0 + R[4] * R[7] * s1 + R[5] * R[8] * s2;
    S[5] = R[6] * R[6] * s0 + R[7] * R[7] * s1 + R[8] * R[8] * s2;
#pragma unroll
    for (int k = 0; k < 6; ++k) g.Sig[k] = (float)S[k];
}

// Camera-space quantities of one Gaussian in one view.
struct ViewProj {
    double tx, ty, tz;     // FP64 camera-space position
    float t[3];            // the same in FP32
    float xt, yt;          // clamped x/z, y/z
    bool clx, cly;         // clamp active
    float T[6];            // J W, 2x3 row-major
    float TS[6];           // T Sigma
    float cov[3];          // Sigma' 00 01 11 (with dilation)
    float conic[3];
    float chol[3];         // Cholesky factor of kappa * conic: l11, l21, l22
};

// Camera-space position; false behind the near plane (or not finite).
__device__ __forceinline__ bool view_position(const gs_camera& c, float near_plane,
                                              const float mu[3], ViewProj& p) {
    const double x = mu[0], y = mu[1], z = mu[2];
    p.tx = fma((double)c.R[0], x, fma((double)c.R[1], y, fma((double)c.R[2], z, (double)c.t[0])));
    p.ty = fma((double)c.R[3], x, fma((double)c.R[4], y, fma((double)c.R[5], z, (double)c.t[1])));
    p.tz = fma((double)c.R[6], x, fma((double)c.R[7], y, fma((double)c.R[8], z, (double)c.t[2])));
    return p.tz > (double)near_plane && isfinite(p.tx) && isfinite(p.ty);
}

// True only when the footprint box { o G >= 1/255 } of the projection below
// certainly holds no pixel centre of the view: its half-widths are bounded
// from above without the screen-space covariance, by
// Sigma'_xx <= |row 0 of J W|^2 lambda_max(Sigma) + dilation, lambda_max(Sigma)
// being the largest squared scale.  Evaluated in FP32 with a relative slack of
// 2^-8, two pixels and 2^-16 of the centre's coordinate, far above the
// rounding of either path (a NaN or an overflow leaves the Gaussian to the
// exact path).  Gaussians that are in front of the camera but off screen then
// skip the FP64 covariance; the outputs do not change, as the exact path
// finds their box empty too.
__device__ __forceinline__ bool surely_off_screen(const gs_camera& c, const gs_view_info& vi,
                                                  const ViewProj& p, const Activated& g) {
    const float tx = (float)p.tx, ty = (float)p.ty, iz = 1.0f / (float)p.tz;
    const float limx = GS_FOV_CLAMP * (0.5f * vi.width / c.fx);
    const float limy = GS_FOV_CLAMP * (0.5f * vi.height / c.fy);
    const float xr = fminf(fmaxf(tx * iz, -limx), limx);
    const float yr = fminf(fmaxf(ty * iz, -limy), limy);
    const float J00 = c.fx * iz, J02 = -c.fx * xr * iz;
    const float J11 = c.fy * iz, J12 = -c.fy * yr * iz;
    float n0 = 0.f, n1 = 0.f;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const float t0 = fmaf(J00, c.R[b], J02 * c.R[6 + b]);
        const float t1 = fmaf(J11, c.R[3 + b], J12 * c.R[6 + b]);
        n0 = fmaf(t0, t0, n0);
        n1 = fmaf(t1, t1, n1);
    }
    const float lam = fmaxf(fmaxf(g.s[0] * g.s[0], g.s[1] * g.s[1]), g.s[2] * g.s[2]);
    const float slack = 1.0f + 1.0f / 256.0f;
    const float L = 2.0f * logf(255.0f * g.o) * slack;
    const float k = (float)GS_FOOTPRINT_INFLATE * slack;
    const float u = fmaf(c.fx, tx * iz, c.cx), w = fmaf(c.fy, ty * iz, c.cy);
    // (the rounding of u and w grows with their magnitude: 2^-16 of it more)
    const float ex = sqrtf(L * fmaf(n0 * lam, slack, GS_DILATION)) * k + 2.0f + fabsf(u) * 0x1p-16f;
    const float ey = sqrtf(L * fmaf(n1 * lam, slack, GS_DILATION)) * k + 2.0f + fabsf(w) * 0x1p-16f;
    return u + ex < 0.5f || u - ex > (float)vi.width - 0.5f || w + ey < 0.5f ||
           w - ey > (float)vi.height - 0.5f;
}

// The rest of the projection of a Gaussian in front of the camera: J, the
// screen-space covariance, its conic and Cholesky factor.
__device__ __forceinline__ void view_shape(const gs_camera& c, const gs_view_info& vi,
                                           const Activated& g, ViewProj& p) {
    p.t[0] = (float)p.tx;
    p.t[1] = (float)p.ty;
    p.t[2] = (float)p.tz;
    const double limx = (double)GS_FOV_CLAMP * (0.5 * vi.width / (double)c.fx);
    const double limy = (double)GS_FOV_CLAMP * (0.5 * vi.height / (double)c.fy);
    double xr = p.tx / p.tz, yr = p.ty / p.tz;
    p.clx = xr < -limx || xr > limx;
    p.cly = yr < -limy || yr > limy;
    xr = xr < -limx ? -limx : (xr > limx ? limx : xr);
    yr = yr < -limy ? -limy : (yr > limy ? limy : yr);
    p.xt = (float)xr;
    p.yt = (float)yr;
    // J W, T Sigma, Sigma' and its inverse in FP64 (see activate_rot), stored as FP32
    const double iz = 1.0 / p.tz;
    const double J00 = c.fx * iz, J02 = -(double)c.fx * xr * iz;
    const double J11 = c.fy * iz, J12 = -(double)c.fy * yr * iz;
    double T[6];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        T[b] = J00 * c.R[b] + J02 * c.R[6 + b];
        T[3 + b] = J11 * c.R[3 + b] + J12 * c.R[6 + b];
    }
    const double* S = g.SigD;
    double TS[6];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const double* Tr = T + 3 * u;
        TS[3 * u + 0] = Tr[0] * S[0] + Tr[1] * S[1] + Tr[2] * S[2];
        TS[3 * u + 1] = Tr[0] * S[1] + Tr[1] * S[3] + Tr[2] * S[4];
        TS[3 * u + 2] = Tr[0] * S[2] + Tr[1] * S[4] + Tr[2] * S[5];
    }
    const double c0 = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2] + (double)GS_DILATION;
    const double c1 = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
    const double c2 = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5] + (double)GS_DILATION;
    const double idet = 1.0 / (c0 * c2 - c1 * c1);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        p.T[k] = (float)T[k];
        p.TS[k] = (float)TS[k];
    }
    p.cov[0] = (float)c0;
    p.cov[1] = (float)c1;
    p.cov[2] = (float)c2;
    p.conic[0] = (float)(c2 * idet);
    p.conic[1] = (float)(-c1 * idet);
    p.conic[2] = (float)(c0 * idet);
    // kappa Q = L L^T: l11 = sqrt(kappa a), l21 = kappa b / l11, l22^2 = kappa det(Q) / a
    // = kappa / Sigma'_yy
    const double kappa = GS_KAPPA_D;
    const double l11 = sqrt(kappa * c2 * idet);
    p.chol[0] = (float)l11;
    p.chol[1] = (float)(-kappa * c1 * idet / l11);
    p.chol[2] = (float)sqrt(kappa / c2);
}

__device__ __forceinline__ bool view_project(const gs_camera& c, const gs_view_info& vi,
                                             float near_plane, const float mu[3],
                                             const Activated& g, ViewProj& p) {
    if (!view_position(c, near_plane, mu, p)) return false;
    view_shape(c, vi, g, p);
    return true;
}

template <int DEG, bool SIGMA3>
__global__ void __launch_bounds__(GS_BLOCK) project_fwd_kernel(ProjArgs a) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (i >= a.n) return;
    const int64_t n = a.n;
    const Raw raw = load_raw(a, i);
    float mu[3];
    Activated g;
    activate_light(raw, mu, g);
    activate_rot(raw, g);

    u32 vis = 0;   // views that bin this Gaussian (bit v)
    for (int v = 0; v < a.V; ++v) {
        const gs_camera c = a.cams[v];
        const gs_view_info vi = a.views[v];
        const int64_t e = (int64_t)v * n + i;
        ViewProj p;
        const bool ok = view_position(c, a.near_plane, mu, p);
        a.depth_key[e] = __float_as_uint((float)p.tz);
        u32 tt = 0;
        uint2 rc = make_uint2(0u, 0u);
        if (ok && (SIGMA3 || (g.o >= GS_ALPHA_MIN && !surely_off_screen(c, vi, p, g)))) {
            view_shape(c, vi, g, p);
            const double u = (double)c.fx * p.tx / p.tz + (double)c.cx;
            const double w = (double)c.fy * p.ty / p.tz + (double)c.cy;
            double x0, x1, y0, y1;   // tile columns and rows, inclusive
            bool nonempty;
            if (SIGMA3) {
                // the tiles whose squares meet [u - r, u + r] x [w - r, w + r],
                // r = ceil(3 sqrt(largest eigenvalue of Sigma'))
                const double s0 = p.cov[0], s1 = p.cov[1], s2 = p.cov[2];
                const double mid = 0.5 * (s0 + s2);
                const double lam = mid + sqrt(fmax(mid * mid - (s0 * s2 - s1 * s1), 0.0));
                const double r = ceil(3.0 * sqrt(lam));
                x0 = ceil((u - r) / GS_TILE) - 1.0;
                x1 = floor((u + r) / GS_TILE);
                y0 = ceil((w - r) / GS_TILE) - 1.0;
                y1 = floor((w + r) / GS_TILE);
                x0 = x0 < 0.0 ? 0.0 : x0;
                y0 = y0 < 0.0 ? 0.0 : y0;
                x1 = x1 > vi.tiles_x - 1 ? (double)(vi.tiles_x - 1) : x1;
                y1 = y1 > vi.tiles_y - 1 ? (double)(vi.tiles_y - 1) : y1;
                nonempty = x0 <= x1 && y0 <= y1;
            } else {
                // footprint: bounding box of { o G >= 1/255 }, inflated by 2^-10
                const float L = 2.0f * logf(255.0f * g.o);
                const double ex = (double)(sqrtf(L * p.cov[0]) * (float)GS_FOOTPRINT_INFLATE);
                const double ey = (double)(sqrtf(L * p.cov[2]) * (float)GS_FOOTPRINT_INFLATE);
                x0 = ceil(u - ex - 0.5);
                x1 = floor(u + ex - 0.5);
                y0 = ceil(w - ey - 0.5);
                y1 = floor(w + ey - 0.5);
                x0 = x0 < 0.0 ? 0.0 : x0;
                y0 = y0 < 0.0 ? 0.0 : y0;
                x1 = x1 > vi.width - 1 ? (double)(vi.width - 1) : x1;
                y1 = y1 > vi.height - 1 ? (double)(vi.height - 1) : y1;
                // some pixel centre inside; then the tiles of those pixels
                nonempty = x0 <= x1 && y0 <= y1;
                x0 = floor(x0 / GS_TILE);
                x1 = floor(x1 / GS_TILE);
                y0 = floor(y0 / GS_TILE);
                y1 = floor(y1 / GS_TILE);
            }
            if (nonempty) {
                const u32 tx0 = (u32)x0, tx1 = (u32)x1;
                const u32 ty0 = (u32)y0, ty1 = (u32)y1;
                rc = make_uint2(tx0 | (tx1 << 16), ty0 | (ty1 << 16));
                const float uh = (float)u, wh = (float)w;
                const float ul = (float)(u - (double)uh), wl = (float)(w - (double)wh);
                const float4 s0 = make_float4(uh, wh, ul, wl);
                const float4 s1 = make_float4(p.chol[0], p.chol[1], p.chol[2], g.o);
                a.splat[3 * e + 0] = s0;
                a.splat[3 * e + 1] = s1;
                if (SIGMA3) {
                    tt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
                } else {
                    // bin to the tiles of the rectangle whose squares meet the ellipse
                    const FootprintRows fr = footprint_rows(s0, s1);
                    int first;
                    for (u32 ty = ty0; ty <= ty1; ++ty)
                        tt += footprint_row_count(fr, (int)ty, (int)tx0, (int)tx1, &first);
                }
            }
        }
        a.tiles_touched[e] = tt;
        if (tt) {
            a.rect[e] = rc;
            vis |= 1u << v;
            // the adjoint of this step accumulates into these
#pragma unroll
            for (int k = 0; k < 9; ++k) a.splat_grad[9 * e + k] = 0.f;
        }
    }
    // colour, for the views that bin the Gaussian: the colour coefficients (192
    // of the 236 bytes of a Gaussian) are read only by lanes that need them, and
    // not at all by a wave with no such lane (whole waves of Gaussians outside
    // every view, when the Gaussians are in spatial order)
    if (__ballot(vis != 0) == 0) return;
    float f[K][3];
    if (vis) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                f[k][ch] = __builtin_nontemporal_load(a.sh + ((int64_t)k * 3 + ch) * n + i);
    }
    for (u32 m = vis; m; m &= m - 1) {
        const int v = __builtin_ctz(m);
        const gs_camera c = a.cams[v];
        const int64_t e = (int64_t)v * n + i;
        float Y[16], dir[3], idist;
        view_basis<DEG>(c, mu, Y, dir, idist);
        float rgb[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float acc = 0.5f;
#pragma unroll
            for (int k = 0; k < K; ++k) acc = fmaf(Y[k], f[k][ch], acc);
            rgb[ch] = acc > 0.f ? acc : 0.f;
        }
        a.splat[3 * e + 2] = make_float4(rgb[0], rgb[1], rgb[2], 0.f);
    }
}

struct ProjBwdArgs {
    ProjArgs p;
    const u32* tiles_touched;
    const float* splat_grad;
    float* d_means;
    float* d_log_scales;
    float* d_quats;
    float* d_logits;
    float* d_sh;
    float* accum;
    float* denom;
    int rendered_only;     // rows of Gaussians no view rendered are not written
    // fused sparse Adam (gs_project_backward_adam) of parameter array k
    // (means, log_scales, quats, logits, sh; ap[k] == nullptr: its gradient is
    // written instead): the parameters and moments, step sizes, decay rates,
    // eps and the bias-correction factors (from the device counter when set)
    float* ap[5];
    float* am[5];
    float* av[5];
    float alr[5];
    float b1, b2, eps, c1, c2;
    const gs_adam_counter* counter;
};

// R rows of the fused sparse Adam step: elements j0 + r n of parameter array
// k, with summed gradients g[r], take the optimiser kernel's update (a
// Gaussian no view rendered stores back what it read, as there); p: their
// values when the caller holds them, else they are read again.  Every load is
// issued before the first update.
template <int R>
__device__ __forceinline__ void fused_adam_rows(const ProjBwdArgs& b, int k, int64_t j0, int64_t n,
                                                bool upd, const float* g, const float* p,
                                                float c1, float c2) {
    float m[R], v[R], q[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j = j0 + r * n;
        m[r] = __builtin_nontemporal_load(b.am[k] + j);
        v[r] = __builtin_nontemporal_load(b.av[k] + j);
        q[r] = p ? p[r] : b.ap[k][j];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j = j0 + r * n;
        adam_element(upd, g[r], m[r], v[r], q[r], b.alr[k], b.b1, b.b2, b.eps, c1, c2);
        __builtin_nontemporal_store(m[r], b.am[k] + j);
        __builtin_nontemporal_store(v[r], b.av[k] + j);
        __builtin_nontemporal_store(q[r], b.ap[k] + j);
    }
}

template <int DEG>
__global__ void __launch_bounds__(GS_BLOCK) project_bwd_kernel(ProjBwdArgs b) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const ProjArgs& a = b.p;
    const int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (i >= a.n) return;
    const int64_t n = a.n;
    // the views that rendered this Gaussian (bit v)
    u32 rend = 0;
    for (int v = 0; v < a.V; ++v) rend |= (b.tiles_touched[(int64_t)v * n + i] != 0 ? 1u : 0u) << v;
    // A wave of Gaussians no view rendered reads nothing more and writes zero
    // gradients, or nothing when only rendered rows are wanted (whole waves of
    // them, when the Gaussians are in spatial order).
    if (__ballot(rend != 0) == 0) {
        // (the fused Adam step leaves such Gaussians as they are, like the
        // optimiser kernel, and writes no gradient for the arrays it covers)
        if (b.rendered_only) return;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (!b.ap[0]) __builtin_nontemporal_store(0.f, b.d_means + k * n + i);
            if (!b.ap[1]) __builtin_nontemporal_store(0.f, b.d_log_scales + k * n + i);
        }
        if (!b.ap[2])
#pragma unroll
            for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(0.f, b.d_quats + k * n + i);
        if (!b.ap[3]) __builtin_nontemporal_store(0.f, b.d_logits + i);
        if (!b.ap[4])
#pragma unroll
            for (int k = 0; k < 3 * K; ++k) __builtin_nontemporal_store(0.f, b.d_sh + (int64_t)k * n + i);
        return;
    }
    // Otherwise every lane of the wave takes the same path (a Gaussian no view
    // rendered just gets zeros): when the rendered Gaussians are scattered over
    // the index order every 128-byte line of the SoA arrays is fetched anyway,
    // and a divergent early exit would split each store into partial-line writes.
    // every load first, so one memory latency covers the parameters and the
    // colour coefficients (the scheduler would otherwise sink the colour loads
    // below the activation arithmetic, serialising two latencies); the colour
    // coefficients, 192 of the 236 bytes, are read once per pass: non-temporal
    float f[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
            f[k][ch] = __builtin_nontemporal_load(a.sh + ((int64_t)k * 3 + ch) * n + i);
    const Raw raw = load_raw(a, i);
    __builtin_amdgcn_sched_barrier(0);
    float mu[3];
    Activated g;
    activate_light(raw, mu, g);
    activate_rot(raw, g);

    float dmu[3] = {0.f, 0.f, 0.f};
    float dls[3] = {0.f, 0.f, 0.f};
    float dq[4] = {0.f, 0.f, 0.f, 0.f};
    float dlogit = 0.f;
    float dsh[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) dsh[k][0] = dsh[k][1] = dsh[k][2] = 0.f;
    float st_acc = 0.f, st_den = 0.f;
    // G R (3x3) and diag(R^T G R) (3) summed over views, G = dL/dSigma; kept
    // instead of G itself (see the per-view update below)
    float GRs[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float RGR[3] = {0.f, 0.f, 0.f};

    for (int v = 0; v < a.V; ++v) {
        const int64_t e = (int64_t)v * n + i;
        if (!((rend >> v) & 1u)) continue;
        const gs_camera c = a.cams[v];
        const gs_view_info vi = a.views[v];
        ViewProj p;
        if (!view_project(c, vi, a.near_plane, mu, g, p)) continue;
        float gr[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) gr[k] = b.splat_grad[9 * e + k];

        // densification statistic: position gradient in NDC units
        {
            const float gx = gr[0] * (0.5f * (float)vi.width);
            const float gy = gr[1] * (0.5f * (float)vi.height);
            st_acc += sqrtf(gx * gx + gy * gy);
            st_den += 1.f;
        }
        // opacity = sigmoid(logit)
        dlogit += gr[5] * g.o * (1.f - g.o);

        // colour = max(0, sum_k Y_k f_k + 1/2), direction from the camera centre
        {
            float Y[16], dir[3], idist;
            view_basis<DEG>(c, mu, Y, dir, idist);
            const float dx = dir[0], dy = dir[1], dz = dir[2];
            float wk[16];
#pragma unroll
            for (int k = 0; k < K; ++k) wk[k] = 0.f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.5f;
#pragma unroll
                for (int k = 0; k < K; ++k) acc = fmaf(Y[k], f[k][ch], acc);
                const float gc = acc < 0.f ? 0.f : gr[6 + ch];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    dsh[k][ch] += Y[k] * gc;
                    wk[k] += f[k][ch] * gc;
                }
            }
            if (DEG > 0) {
                float gdx, gdy, gdz;
                sh_grad_contract<DEG>(dx, dy, dz, wk, gdx, gdy, gdz);
                const float dd = dx * gdx + dy * gdy + dz * gdz;
                dmu[0] += (gdx - dx * dd) * idist;
                dmu[1] += (gdy - dy * dd) * idist;
                dmu[2] += (gdz - dz * dd) * idist;
            }
        }

        // conic -> Sigma': G_Sigma' = -Q G_Q Q with G_Q = [[ga, gb/2], [gb/2, gc]]
        const float qa = p.conic[0], qb = p.conic[1], qc = p.conic[2];
        const float ga = gr[2], gb = 0.5f * gr[3], gc = gr[4];
        const float P00 = qa * ga + qb * gb, P01 = qa * gb + qb * gc;
        const float P10 = qb * ga + qc * gb, P11 = qb * gb + qc * gc;
        const float S00 = -(P00 * qa + P01 * qb);
        const float S01 = -0.5f * ((P00 * qb + P01 * qc) + (P10 * qa + P11 * qb));
        const float S11 = -(P10 * qb + P11 * qc);
        // Sigma' = T Sigma T^T + 0.3 I: G_Sigma = T^T S T, G_T = 2 S T Sigma.
        // The scale and rotation gradients only need G R and diag(R^T G R),
        // taken here through the Gaussian's axes projected to the screen,
        // v_k = T R_k, and u_k = Q v_k:  S v_k = -Q (G_Q u_k), so
        // G R_k = T^T S v_k and R_k^T G R_k = -u_k . (G_Q u_k).  Neither G nor
        // S is contracted with an axis directly: G has a null direction (the
        // ray; T is 2x3), and S = -Q G_Q Q applied to an axis along the long
        // side of the ellipse (near Q's small eigenvector) cancels by the square
        // of Sigma's eigenvalue ratio, leaving FP32 rounding far above the result.
        const float* T = p.T;
        {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float v0 = T[0] * g.R[k] + T[1] * g.R[3 + k] + T[2] * g.R[6 + k];
                const float v1 = T[3] * g.R[k] + T[4] * g.R[3 + k] + T[5] * g.R[6 + k];
                const float u0 = qa * v0 + qb * v1, u1 = qb * v0 + qc * v1;
                const float z0 = ga * u0 + gb * u1, z1 = gb * u0 + gc * u1;
                RGR[k] -= u0 * z0 + u1 * z1;
                const float w0 = -(qa * z0 + qb * z1), w1 = -(qb * z0 + qc * z1);
#pragma unroll
                for (int r = 0; r < 3; ++r) GRs[3 * r + k] += T[r] * w0 + T[3 + r] * w1;
            }
        }
        float GT[6];
        {
            const float* TS = p.TS;  // (T Sigma)
            GT[0] = 2.f * (S00 * TS[0] + S01 * TS[3]);
            GT[1] = 2.f * (S00 * TS[1] + S01 * TS[4]);
            GT[2] = 2.f * (S00 * TS[2] + S01 * TS[5]);
            GT[3] = 2.f * (S01 * TS[0] + S11 * TS[3]);
            GT[4] = 2.f * (S01 * TS[1] + S11 * TS[4]);
            GT[5] = 2.f * (S01 * TS[2] + S11 * TS[5]);
        }
        // T = J W:  G_J = G_T W^T (only J00, J02, J11, J12 vary)
        const float* W = c.R;
        const float GJ00 = GT[0] * W[0] + GT[1] * W[1] + GT[2] * W[2];
        const float GJ02 = GT[0] * W[6] + GT[1] * W[7] + GT[2] * W[8];
        const float GJ11 = GT[3] * W[3] + GT[4] * W[4] + GT[5] * W[5];
        const float GJ12 = GT[3] * W[6] + GT[4] * W[7] + GT[5] * W[8];
        const float tz = p.t[2], iz = 1.0f / tz, iz2 = iz * iz;
        float gt0 = 0.f, gt1 = 0.f, gt2 = 0.f;
        gt2 -= (GJ00 * c.fx + GJ11 * c.fy) * iz2;
        if (!p.clx) {
            gt0 -= GJ02 * c.fx * iz2;
            gt2 += GJ02 * 2.f * c.fx * p.t[0] * iz2 * iz;
        } else {
            gt2 += GJ02 * c.fx * p.xt * iz2;
        }
        if (!p.cly) {
            gt1 -= GJ12 * c.fy * iz2;
            gt2 += GJ12 * 2.f * c.fy * p.t[1] * iz2 * iz;
        } else {
            gt2 += GJ12 * c.fy * p.yt * iz2;
        }
        // mean2d = (fx tx/tz + cx, fy ty/tz + cy)
        gt0 += gr[0] * c.fx * iz;
        gt1 += gr[1] * c.fy * iz;
        gt2 -= (gr[0] * c.fx * p.t[0] + gr[1] * c.fy * p.t[1]) * iz2;
        // t = W mu + t_w
        dmu[0] += W[0] * gt0 + W[3] * gt1 + W[6] * gt2;
        dmu[1] += W[1] * gt0 + W[4] * gt1 + W[7] * gt2;
        dmu[2] += W[2] * gt0 + W[5] * gt1 + W[8] * gt2;
    }

    // Sigma = M M^T, M = R diag(s):  G_M = 2 G M, so dL/dR = G_M diag(s) =
    // 2 (G R) diag(s^2) and dL/dlog s_k = s_k (R^T G_M)_kk = 2 s_k^2 R_k^T G R_k
    {
        float GR[9];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float s2 = 2.f * g.s[k] * g.s[k];
#pragma unroll
            for (int r = 0; r < 3; ++r) GR[3 * r + k] = GRs[3 * r + k] * s2;
            dls[k] = RGR[k] * s2;
        }
        // dL/dR -> unit quaternion -> raw quaternion (the tangent projection
        // (I - q q^T) / |q|), in FP64 from the raw quaternion: the projection
        // cancels the radial part, which can be most of the unit-quaternion
        // gradient
        const double q0 = raw.q[0], q1 = raw.q[1], q2 = raw.q[2], q3 = raw.q[3];
        const double iq = 1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
        const double w = q0 * iq, x = q1 * iq, y = q2 * iq, z = q3 * iq;
        double G[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) G[k] = GR[k];
        const double gw = 2.0 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
        const double gx = 2.0 * (y * G[1] + z * G[2] + y * G[3] - 2.0 * x * G[4] - w * G[5] +
                                 z * G[6] + w * G[7] - 2.0 * x * G[8]);
        const double gy = 2.0 * (-2.0 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] -
                                 w * G[6] + z * G[7] - 2.0 * y * G[8]);
        const double gz = 2.0 * (-2.0 * z * G[0] - w * G[1] + x * G[2] + w * G[3] -
                                 2.0 * z * G[4] + y * G[5] + x * G[6] + y * G[7]);
        const double dot = w * gw + x * gx + y * gy + z * gz;
        dq[0] = (float)((gw - w * dot) * iq);
        dq[1] = (float)((gx - x * dot) * iq);
        dq[2] = (float)((gy - y * dot) * iq);
        dq[3] = (float)((gz - z * dot) * iq);
    }

    // Gradients and colour coefficients stream through once: non-temporal
    // stores and loads keep them from evicting the step's reused data and leave
    // no dirty lines for the next kernel to write back.
    // Each array's summed gradient goes to HBM, or straight into its fused
    // sparse Adam step (the parameter itself reread: its line is in the cache,
    // and keeping it live across the view loop would cost registers; the
    // colour coefficients are still held).
    float c1 = b.c1, c2 = b.c2;
    if (b.counter) {
        const int64_t t = b.counter->step + 1;
        c1 = adam_bias_factor(b.b1, t);
        c2 = adam_bias_factor(b.b2, t);
    }
    const bool upd = rend != 0;
    if (b.ap[0]) {
        fused_adam_rows<3>(b, 0, i, n, upd, dmu, nullptr, c1, c2);
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) __builtin_nontemporal_store(dmu[k], b.d_means + k * n + i);
    }
    if (b.ap[1]) {
        fused_adam_rows<3>(b, 1, i, n, upd, dls, nullptr, c1, c2);
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) __builtin_nontemporal_store(dls[k], b.d_log_scales + k * n + i);
    }
    if (b.ap[2]) {
        fused_adam_rows<4>(b, 2, i, n, upd, dq, nullptr, c1, c2);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(dq[k], b.d_quats + k * n + i);
    }
    if (b.ap[3]) fused_adam_rows<1>(b, 3, i, n, upd, &dlogit, nullptr, c1, c2);
    else __builtin_nontemporal_store(dlogit, b.d_logits + i);
    if (b.ap[4]) {
        // a coefficient's three channels at a time (their values are held)
#pragma unroll
        for (int k = 0; k < K; ++k) fused_adam_rows<3>(b, 4, (int64_t)k * 3 * n + i, n, upd, dsh[k],
                                                       f[k], c1, c2);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch)
                __builtin_nontemporal_store(dsh[k][ch], b.d_sh + ((int64_t)k * 3 + ch) * n + i);
    }
    if (b.accum) {
        b.accum[i] += st_acc;
        b.denom[i] += st_den;
    }
}

ProjArgs make_args(gs_frame* f, const gs_gaussians* g, const gs_camera* cams, float near_plane) {
    ProjArgs a;
    a.means = g->means;
    a.log_scales = g->log_scales;
    a.quats = g->quats;
    a.logits = g->opacity_logits;
    a.sh = g->sh;
    a.n = g->n;
    a.V = f->V;
    a.near_plane = near_plane;
    a.cams = cams;
    a.views = f->d_views;
    a.depth_key = f->depth_key;
    a.tiles_touched = f->tiles_touched;
    a.rect = f->rect;
    a.splat = f->splat;
    a.splat_grad = f->splat_grad;
    return a;
}

}  // namespace

template <bool SIGMA3>
void launch_project_fwd(const ProjArgs& a, int sh_degree, unsigned blocks, hipStream_t s) {
    switch (sh_degree) {
        case 0: project_fwd_kernel<0, SIGMA3><<<blocks, GS_BLOCK, 0, s>>>(a); break;
        case 1: project_fwd_kernel<1, SIGMA3><<<blocks, GS_BLOCK, 0, s>>>(a); break;
        case 2: project_fwd_kernel<2, SIGMA3><<<blocks, GS_BLOCK, 0, s>>>(a); break;
        default: project_fwd_kernel<3, SIGMA3><<<blocks, GS_BLOCK, 0, s>>>(a); break;
    }
}

gs_status gs_launch_project(gs_frame* f, const gs_gaussians* g, const gs_camera* cams,
                            float near_plane, bool sigma3, hipStream_t s) {
    f->sigma3 = sigma3;
    if (f->n == 0) return GS_OK;
    ProjArgs a = make_args(f, g, cams, near_plane);
    const unsigned blocks = (unsigned)((f->n + GS_BLOCK - 1) / GS_BLOCK);
    if (sigma3) launch_project_fwd<true>(a, g->sh_degree, blocks, s);
    else launch_project_fwd<false>(a, g->sh_degree, blocks, s);
    return gs_check_launch("project_fwd");
}

gs_status gs_launch_project_bwd(gs_frame* f, const gs_gaussians* g, const gs_camera* cams,
                                float near_plane, const gs_gaussian_grads* gr, float* accum,
                                float* denom, bool rendered_only, const gs_fused_adam* adam,
                                hipStream_t s) {
    if (f->n == 0) return GS_OK;
    ProjBwdArgs b;
    b.p = make_args(f, g, cams, near_plane);
    b.tiles_touched = f->tiles_touched;
    b.splat_grad = f->splat_grad;
    b.d_means = gr->means;
    b.d_log_scales = gr->log_scales;
    b.d_quats = gr->quats;
    b.d_logits = gr->opacity_logits;
    b.d_sh = gr->sh;
    b.accum = accum;
    b.denom = denom;
    b.rendered_only = rendered_only ? 1 : 0;
    b.b1 = b.b2 = b.eps = 0.f;
    b.c1 = b.c2 = 1.f;
    b.counter = nullptr;
    for (int k = 0; k < 5; ++k) {
        b.ap[k] = adam ? adam->param[k] : nullptr;
        b.am[k] = adam ? adam->m[k] : nullptr;
        b.av[k] = adam ? adam->v[k] : nullptr;
        b.alr[k] = adam ? adam->lr[k] : 0.f;
    }
    if (adam) {
        b.b1 = adam->beta1;
        b.b2 = adam->beta2;
        b.eps = adam->eps;
        b.counter = adam->counter;
        if (!adam->counter) {
            b.c1 = adam_bias_factor(adam->beta1, adam->step);
            b.c2 = adam_bias_factor(adam->beta2, adam->step);
        }
    }
    const unsigned blocks = (unsigned)((f->n + GS_BLOCK - 1) / GS_BLOCK);
    switch (g->sh_degree) {
        case 0: project_bwd_kernel<0><<<blocks, GS_BLOCK, 0, s>>>(b); break;
        case 1: project_bwd_kernel<1><<<blocks, GS_BLOCK, 0, s>>>(b); break;
        case 2: project_bwd_kernel<2><<<blocks, GS_BLOCK, 0, s>>>(b); break;
        default: project_bwd_kernel<3><<<blocks, GS_BLOCK, 0, s>>>(b); break;
    }
    return gs_check_launch("project_bwd");
}
