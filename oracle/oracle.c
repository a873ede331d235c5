/*
 * FP64 CPU oracle for Gaussian-splatting rendering, its adjoint and
 * densification.  TEST INFRASTRUCTURE ONLY: this file is compiled and called
 * by the test-suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  The GPU library never links, includes or calls it, and it never
 * includes anything from the GPU library.
 *
 * It is deliberately plain and slow: every pixel looks at every Gaussian, no
 * tiles, no binning, no blocking, in double precision.  Each routine cites
 * the passage of the paper it follows ("Decomposing Densification in Gaussian
 * Splatting for Faster 3D Scene Reconstruction"):
 *   - Gaussian primitive and covariance Sigma = R S S^T R^T: Preliminary, Eq. 1.
 *   - Screen-space covariance Sigma' = J W Sigma W^T J^T: Preliminary.
 *   - Alpha compositing of depth-sorted Gaussians, sigma_i = alpha_i G'_i(p): Eq. 2.
 *   - Colour c_i evaluated from spherical harmonics: Preliminary / Eq. 2.
 *   - Densification statistic and split/clone rule: Preliminary, last paragraph.
 *   - Adaptive opacity threshold tau = min(alpha_sorted[floor(N p)], tau_u):
 *     Methodology, Adaptive Opacity Pruning.
 * Points the paper leaves open are fixed as follows (same constants as the
 * GPU library, as FP32 values widened to double):
 *   alpha = min(0.99, o G); a Gaussian with alpha < 1/255 is skipped; the walk
 *   stops before compositing a Gaussian that would bring T below 1e-4;
 *   pixel (px,py) is sampled at (px+0.5, py+0.5); Sigma' gets +0.3 px^2 on its
 *   diagonal; x/z and y/z are clamped to +-1.3 tan(half fov) inside J only;
 *   Gaussians with camera depth <= near (0.2) are culled; the footprint of a
 *   Gaussian is the bounding box of the ellipse o G >= 1/255 inflated by 2^-10,
 *   and it is binned to the tiles of that box whose square meets the ellipse;
 *   depth order uses the FP32 rounding of the camera depth (computed as a
 *   fused multiply-add chain in double), ties broken by Gaussian index;
 *   real spherical harmonics with the Condon-Shortley phase, rgb = max(0, sum + 1/2).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ALPHA_MAX ((double)0.99f)
#define ALPHA_MIN ((double)(1.0f / 255.0f))
#define T_MIN ((double)1e-4f)
#define DILATION ((double)0.3f)
#define FOV_CLAMP 1.3
#define FOOTPRINT_INFLATE (1.0 + 1.0 / 1024.0)
#define TILE 16

/* ------------------------------------------------------------------------ */
/* Spherical harmonics from the definition                                    */
/* ------------------------------------------------------------------------ */
/* Real SH with the Condon-Shortley phase, index k = l*l + l + m, m = -l..l:
 *   m > 0: sqrt(2) K_lm P_l^m(cos th) cos(m ph)
 *   m < 0: sqrt(2) K_l|m| P_l^|m|(cos th) sin(|m| ph)
 *   m = 0: K_l0 P_l(cos th)
 * K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), P_l^m(x) = (-1)^m (1-x^2)^(m/2) d^m P_l/dx^m.
 * On the unit sphere (1-z^2)^(m/2) {cos, sin}(m ph) = {Re, Im}((x + i y)^m), which
 * turns every Y into a polynomial in (x, y, z); its gradient is used for the
 * direction derivative (the caller projects it onto the tangent plane).      */

#define SH_MAXL 3
static double legendre_coef[SH_MAXL + 1][SH_MAXL + 1]; /* P_l(x) = sum_j c[l][j] x^j */
static int legendre_ready = 0;

/* Built once when the library loads, before any OpenMP region can reach it
 * (a lazy first-use build raced with readers on other threads). */
__attribute__((constructor)) static void legendre_init(void) {
    if (legendre_ready) return;
    memset(legendre_coef, 0, sizeof(legendre_coef));
    legendre_coef[0][0] = 1.0;
    legendre_coef[1][1] = 1.0;
    /* (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1} */
    for (int l = 1; l < SH_MAXL; ++l) {
        for (int j = 0; j <= SH_MAXL; ++j) {
            double v = 0.0;
            if (j >= 1) v += (2 * l + 1) * legendre_coef[l][j - 1];
            v -= l * legendre_coef[l - 1][j];
            legendre_coef[l + 1][j] = v / (l + 1);
        }
    }
    legendre_ready = 1;
}

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* Q(z) = d^m P_l / dz^m and its z-derivative. */
static void legendre_dm(int l, int m, double z, double* q, double* dq) {
    double c[SH_MAXL + 1];
    for (int j = 0; j <= SH_MAXL; ++j) c[j] = legendre_coef[l][j];
    for (int d = 0; d < m; ++d) {
        for (int j = 0; j < SH_MAXL; ++j) c[j] = c[j + 1] * (j + 1);
        c[SH_MAXL] = 0.0;
    }
    double v = 0.0, dv = 0.0, zp = 1.0;
    for (int j = 0; j <= SH_MAXL; ++j) {
        v += c[j] * zp;
        zp *= z;
    }
    zp = 1.0;
    for (int j = 1; j <= SH_MAXL; ++j) {
        dv += j * c[j] * zp;
        zp *= z;
    }
    *q = v;
    *dq = dv;
}

/* Y[k] and dY[k][3] = gradient of the polynomial form w.r.t. (x, y, z). */
void oracle_sh_basis(int deg, const double dir[3], double* Y, double* dY) {
    legendre_init();
    const double x = dir[0], y = dir[1], z = dir[2];
    for (int l = 0; l <= deg; ++l) {
        for (int m = -l; m <= l; ++m) {
            const int am = m < 0 ? -m : m;
            const int k = l * l + l + m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double q, dq;
            legendre_dm(l, am, z, &q, &dq);
            /* (x + i y)^am and its derivative am (x + i y)^(am-1) */
            double re = 1.0, im = 0.0, dre = 0.0, dim = 0.0;
            for (int j = 0; j < am; ++j) {
                dre = re;
                dim = im; /* holds (x+iy)^j after loop: derivative uses power am-1 */
                double nre = re * x - im * y, nim = re * y + im * x;
                re = nre;
                im = nim;
            }
            /* dre/dim now hold (x+iy)^(am-1) (or 0 if am == 0) */
            double dpx_re = am * dre, dpx_im = am * dim;   /* d/dx (x+iy)^am */
            double dpy_re = -am * dim, dpy_im = am * dre;  /* d/dy = i * am (x+iy)^(am-1) */
            double A, dAx, dAy;
            if (m > 0) { A = re; dAx = dpx_re; dAy = dpy_re; }
            else if (m < 0) { A = im; dAx = dpx_im; dAy = dpy_im; }
            else { A = 1.0; dAx = 0.0; dAy = 0.0; }
            double cs = (am % 2) ? -1.0 : 1.0;
            double norm = (m == 0) ? K : sqrt(2.0) * K * cs;
            Y[k] = norm * q * A;
            if (dY) {
                dY[3 * k + 0] = norm * q * dAx;
                dY[3 * k + 1] = norm * q * dAy;
                dY[3 * k + 2] = norm * dq * A;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Camera and projection (Preliminary: Sigma, Sigma' = J W Sigma W^T J^T)     */
/* ------------------------------------------------------------------------ */
/* cam[16] = R (row-major 3x3, world->camera), t (3), fx, fy, cx, cy. */

static void quat_to_rot(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* dR[i]/dq_c for the 9 entries of R (unit-quaternion formula), c = 0..3 (w,x,y,z) */
static void quat_to_rot_grad(const double q[4], const double gR[9], double gq[4]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    /* entries of R and their partials */
    double dw = 0, dx = 0, dy = 0, dz = 0;
    /* R00 = 1 - 2y^2 - 2z^2 */
    dy += gR[0] * (-4 * y); dz += gR[0] * (-4 * z);
    /* R01 = 2xy - 2wz */
    dx += gR[1] * 2 * y; dy += gR[1] * 2 * x; dw += gR[1] * (-2 * z); dz += gR[1] * (-2 * w);
    /* R02 = 2xz + 2wy */
    dx += gR[2] * 2 * z; dz += gR[2] * 2 * x; dw += gR[2] * 2 * y; dy += gR[2] * 2 * w;
    /* R10 = 2xy + 2wz */
    dx += gR[3] * 2 * y; dy += gR[3] * 2 * x; dw += gR[3] * 2 * z; dz += gR[3] * 2 * w;
    /* R11 = 1 - 2x^2 - 2z^2 */
    dx += gR[4] * (-4 * x); dz += gR[4] * (-4 * z);
    /* R12 = 2yz - 2wx */
    dy += gR[5] * 2 * z; dz += gR[5] * 2 * y; dw += gR[5] * (-2 * x); dx += gR[5] * (-2 * w);
    /* R20 = 2xz - 2wy */
    dx += gR[6] * 2 * z; dz += gR[6] * 2 * x; dw += gR[6] * (-2 * y); dy += gR[6] * (-2 * w);
    /* R21 = 2yz + 2wx */
    dy += gR[7] * 2 * z; dz += gR[7] * 2 * y; dw += gR[7] * 2 * x; dx += gR[7] * 2 * w;
    /* R22 = 1 - 2x^2 - 2y^2 */
    dx += gR[8] * (-4 * x); dy += gR[8] * (-4 * y);
    gq[0] = dw; gq[1] = dx; gq[2] = dy; gq[3] = dz;
}

typedef struct {
    /* raw parameters (widened) */
    double mu[3], ls[3], q[4], logit;
    /* activated */
    double s[3], qn[4], qnorm, o, R[9], Sigma[9];
    /* camera space */
    double t[3], xt, yt; int clampx, clampy;
    double J[6], T[6], cov2d[3], conic[3], mean2d[2];
    double dir[3], dist;
    double rgb[3], rgb_pre[3];
    int culled;
} proj_t;

static void mat3_mul(const double* A, const double* B, double* C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double v = 0;
            for (int k = 0; k < 3; ++k) v += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = v;
        }
}

static void project_one(int64_t i, int64_t n, int deg, const float* means, const float* log_scales,
                        const float* quats, const float* logits, const float* sh, const double* cam,
                        int W, int H, double near_plane, proj_t* p) {
    memset(p, 0, sizeof(*p));
    for (int c = 0; c < 3; ++c) p->mu[c] = means[c * n + i];
    for (int c = 0; c < 3; ++c) p->ls[c] = log_scales[c * n + i];
    for (int c = 0; c < 4; ++c) p->q[c] = quats[c * n + i];
    p->logit = logits[i];
    for (int c = 0; c < 3; ++c) p->s[c] = exp(p->ls[c]);
    p->qnorm = sqrt(p->q[0] * p->q[0] + p->q[1] * p->q[1] + p->q[2] * p->q[2] + p->q[3] * p->q[3]);
    for (int c = 0; c < 4; ++c) p->qn[c] = p->q[c] / p->qnorm;
    p->o = 1.0 / (1.0 + exp(-p->logit));
    quat_to_rot(p->qn, p->R);
    /* Sigma = R S S^T R^T  (Eq. 1) */
    double M[9], Mt[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = p->R[3 * a + b] * p->s[b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Mt[3 * a + b] = M[3 * b + a];
    mat3_mul(M, Mt, p->Sigma);

    const double* Rw = cam;
    const double* tw = cam + 9;
    const double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    p->t[0] = Rw[0] * p->mu[0] + Rw[1] * p->mu[1] + Rw[2] * p->mu[2] + tw[0];
    p->t[1] = Rw[3] * p->mu[0] + Rw[4] * p->mu[1] + Rw[5] * p->mu[2] + tw[1];
    /* depth as a fused chain: the same rounding as the sort key definition */
    p->t[2] = fma(Rw[6], p->mu[0], fma(Rw[7], p->mu[1], fma(Rw[8], p->mu[2], tw[2])));
    if (!(p->t[2] > near_plane) || !isfinite(p->t[0]) || !isfinite(p->t[1])) {
        p->culled = 1;
        return;
    }
    const double tz = p->t[2];
    const double limx = FOV_CLAMP * (0.5 * W / fx), limy = FOV_CLAMP * (0.5 * H / fy);
    double xr = p->t[0] / tz, yr = p->t[1] / tz;
    p->clampx = (xr < -limx || xr > limx);
    p->clampy = (yr < -limy || yr > limy);
    p->xt = xr < -limx ? -limx : (xr > limx ? limx : xr);
    p->yt = yr < -limy ? -limy : (yr > limy ? limy : yr);
    /* J: Jacobian of the perspective map at t, with clamped x/z, y/z */
    p->J[0] = fx / tz; p->J[1] = 0;       p->J[2] = -fx * p->xt / tz;
    p->J[3] = 0;       p->J[4] = fy / tz; p->J[5] = -fy * p->yt / tz;
    /* T = J W */
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0;
            for (int k = 0; k < 3; ++k) v += p->J[3 * a + k] * Rw[3 * k + b];
            p->T[3 * a + b] = v;
        }
    /* Sigma' = T Sigma T^T + 0.3 I */
    double TS[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0;
            for (int k = 0; k < 3; ++k) v += p->T[3 * a + k] * p->Sigma[3 * k + b];
            TS[3 * a + b] = v;
        }
    double C2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double v = 0;
            for (int k = 0; k < 3; ++k) v += TS[3 * a + k] * p->T[3 * b + k];
            C2[2 * a + b] = v;
        }
    p->cov2d[0] = C2[0] + DILATION;
    p->cov2d[1] = 0.5 * (C2[1] + C2[2]);
    p->cov2d[2] = C2[3] + DILATION;
    const double det = p->cov2d[0] * p->cov2d[2] - p->cov2d[1] * p->cov2d[1];
    p->conic[0] = p->cov2d[2] / det;
    p->conic[1] = -p->cov2d[1] / det;
    p->conic[2] = p->cov2d[0] / det;
    p->mean2d[0] = fx * p->t[0] / tz + cx;
    p->mean2d[1] = fy * p->t[1] / tz + cy;

    /* colour from SH at the viewing direction (mu - camera centre) */
    double cc[3];
    for (int a = 0; a < 3; ++a) cc[a] = -(Rw[a] * tw[0] + Rw[3 + a] * tw[1] + Rw[6 + a] * tw[2]);
    double d[3] = {p->mu[0] - cc[0], p->mu[1] - cc[1], p->mu[2] - cc[2]};
    p->dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) p->dir[a] = d[a] / p->dist;
    const int K = (deg + 1) * (deg + 1);
    double Y[16];
    oracle_sh_basis(deg, p->dir, Y, NULL);
    for (int ch = 0; ch < 3; ++ch) {
        double v = 0.5;
        for (int k = 0; k < K; ++k) v += Y[k] * sh[((int64_t)k * 3 + ch) * n + i];
        p->rgb_pre[ch] = v;
        p->rgb[ch] = v > 0 ? v : 0;
    }
}

/* Footprint rectangle in tiles: bounding box of {p : o G(p) >= 1/255}
 * (pixel centres), inflated by 2^-10, clipped to the image.  Returns 0 when empty. */
static int footprint_rect(const proj_t* p, int W, int H, double shrink, int rect[4]) {
    if (p->culled || p->o < ALPHA_MIN) return 0;
    const double L = 2.0 * log(255.0 * p->o);
    const double ex = sqrt(L * p->cov2d[0]) * FOOTPRINT_INFLATE + shrink;
    const double ey = sqrt(L * p->cov2d[2]) * FOOTPRINT_INFLATE + shrink;
    double x0 = ceil(p->mean2d[0] - ex - 0.5), x1 = floor(p->mean2d[0] + ex - 0.5);
    double y0 = ceil(p->mean2d[1] - ey - 0.5), y1 = floor(p->mean2d[1] + ey - 0.5);
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > W - 1) x1 = W - 1;
    if (y1 > H - 1) y1 = H - 1;
    if (x0 > x1 || y0 > y1) return 0;
    rect[0] = (int)x0 / TILE;
    rect[1] = (int)x1 / TILE;
    rect[2] = (int)y0 / TILE;
    rect[3] = (int)y1 / TILE;
    return 1;
}

/*
 * Project every Gaussian for one camera.  Outputs (per Gaussian i):
 *   mean2d[2n] (x then y, interleaved per i), conic[3n] (a, b, c of Sigma'^-1),
 *   cov2d[3n], opacity[n], rgb[3n], depth[n] (double camera z),
 *   depth_key[n] (bits of the FP32 rounding of depth), visible[n] (1 if the
 *   footprint is non-empty), rect[4n] (tile x0, x1, y0, y1 inclusive),
 *   flags[n]: bit0 = a rect/visibility decision changes within +-1e-3 px of the
 *   footprint bound, bit1 = opacity within 1e-6 of 1/255 or depth within 1e-6 of near.
 */
void oracle_project(int64_t n, int deg, const float* means, const float* log_scales,
                    const float* quats, const float* logits, const float* sh, const double* cam,
                    int W, int H, double near_plane, double* mean2d, double* conic, double* cov2d,
                    double* opacity, double* rgb, double* depth, uint32_t* depth_key,
                    int32_t* visible, int32_t* rect, int32_t* flags) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        proj_t p;
        project_one(i, n, deg, means, log_scales, quats, logits, sh, cam, W, H, near_plane, &p);
        int r[4] = {0, -1, 0, -1};
        int vis = footprint_rect(&p, W, H, 0.0, r);
        int fl = 0;
        if (!p.culled) {
            int ra[4] = {0, -1, 0, -1}, rb[4] = {0, -1, 0, -1};
            double e = 1e-3;
            int va = footprint_rect(&p, W, H, -e, ra), vb = footprint_rect(&p, W, H, e, rb);
            /* shifting the centre as well as the extent */
            proj_t q = p;
            int rc[4] = {0, -1, 0, -1}, rd[4] = {0, -1, 0, -1};
            q.mean2d[0] += e; q.mean2d[1] += e;
            int vc = footprint_rect(&q, W, H, 0.0, rc);
            q.mean2d[0] -= 2 * e; q.mean2d[1] -= 2 * e;
            int vd = footprint_rect(&q, W, H, 0.0, rd);
            if (va != vis || vb != vis || vc != vis || vd != vis ||
                (vis && (memcmp(ra, r, sizeof r) || memcmp(rb, r, sizeof r) ||
                         memcmp(rc, r, sizeof r) || memcmp(rd, r, sizeof r))))
                fl |= 1;
            if (fabs(p.o - ALPHA_MIN) < 1e-6 * ALPHA_MIN) fl |= 2;
        }
        if (fabs(p.t[2] - near_plane) < 1e-6) fl |= 2;
        mean2d[2 * i] = p.mean2d[0];
        mean2d[2 * i + 1] = p.mean2d[1];
        for (int c = 0; c < 3; ++c) {
            conic[3 * i + c] = p.conic[c];
            cov2d[3 * i + c] = p.cov2d[c];
            rgb[3 * i + c] = p.rgb[c];
        }
        opacity[i] = p.o;
        depth[i] = p.t[2];
        float df = (float)p.t[2];
        memcpy(&depth_key[i], &df, 4);
        visible[i] = p.culled ? 0 : vis;
        for (int c = 0; c < 4; ++c) rect[4 * i + c] = r[c];
        flags[i] = fl;
    }
}

/* ------------------------------------------------------------------------ */
/* Per-pixel compositing, Eq. 2                                               */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t key; int32_t idx; double alpha, G; int clamped; } cand_t;

static int cand_cmp(const void* a, const void* b) {
    const cand_t* x = (const cand_t*)a;
    const cand_t* y = (const cand_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Candidates N_p of pixel p: Gaussians not culled with o G(p) >= 1/255, in
 * (depth key, index) order.  Returns the count; *margin gets the smallest
 * relative distance of any alpha to the 1/255 cutoff or the 0.99 clamp. */
static int64_t pixel_candidates(int64_t n, const double* mean2d, const double* conic,
                                const double* opacity, const uint32_t* depth_key,
                                const int32_t* visible, double px, double py, cand_t* out,
                                double* margin) {
    int64_t m = 0;
    double mg = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        if (!visible[i]) continue;
        const double dx = px - mean2d[2 * i], dy = py - mean2d[2 * i + 1];
        const double a = conic[3 * i], b = conic[3 * i + 1], c = conic[3 * i + 2];
        const double power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy;
        if (power < -30.0) continue; /* o G < e^-30 << 1/255: not a candidate */
        const double G = exp(power);
        const double raw = opacity[i] * G;
        const double r1 = fabs(raw - ALPHA_MIN) / ALPHA_MIN;
        if (r1 < mg) mg = r1;
        if (raw < ALPHA_MIN) continue;
        const double r2 = fabs(raw - ALPHA_MAX) / ALPHA_MAX;
        if (r2 < mg) mg = r2;
        out[m].key = depth_key[i];
        out[m].idx = (int32_t)i;
        out[m].G = G;
        out[m].clamped = raw > ALPHA_MAX;
        out[m].alpha = raw > ALPHA_MAX ? ALPHA_MAX : raw;
        ++m;
    }
    qsort(out, (size_t)m, sizeof(cand_t), cand_cmp);
    *margin = mg;
    return m;
}

/* Forward for a list of pixels (pix[2k], pix[2k+1] = px, py).  Per pixel:
 * color[3], T_final, n_comp (number composited), margin (min relative
 * distance of any discrete decision: alpha cutoff/clamp, transmittance stop). */
void oracle_render_pixels(int64_t n, const double* mean2d, const double* conic,
                          const double* opacity, const double* rgb, const uint32_t* depth_key,
                          const int32_t* visible, int64_t npix, const int32_t* pix,
                          const double* bg, double* color, double* T_final, int32_t* n_comp,
                          double* margin) {
#pragma omp parallel
    {
        cand_t* cand = (cand_t*)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < npix; ++k) {
            double mg;
            const double px = pix[2 * k] + 0.5, py = pix[2 * k + 1] + 0.5;
            int64_t m = pixel_candidates(n, mean2d, conic, opacity, depth_key, visible, px, py, cand, &mg);
            double T = 1.0, C[3] = {0, 0, 0};
            int32_t used = 0;
            for (int64_t j = 0; j < m; ++j) {
                const double al = cand[j].alpha;
                const double Tn = T * (1.0 - al);
                const double r3 = fabs(Tn - T_MIN) / T_MIN;
                if (r3 < mg) mg = r3;
                if (Tn < T_MIN) break;
                const int32_t i = cand[j].idx;
                for (int c = 0; c < 3; ++c) C[c] += rgb[3 * i + c] * al * T;
                T = Tn;
                ++used;
            }
            for (int c = 0; c < 3; ++c) color[3 * k + c] = C[c] + T * bg[c];
            T_final[k] = T;
            n_comp[k] = used;
            margin[k] = mg;
        }
        free(cand);
    }
}

/* Adjoint of the compositing for a list of pixels.  dL_dC[3k..] is the
 * loss gradient of pixel k.  Accumulates into per-Gaussian arrays (n x 9):
 *   [0..1] dL/dmean2d, [2..4] dL/d(conic a, b, c) with b the off-diagonal
 *   entry taken once, [5] dL/dopacity, [6..8] dL/drgb,
 * and g_abs (n x 9) receives, for every element, the sum over pixels of the
 * magnitudes of the terms that make it up, with dL/dalpha and Q d expanded into
 * their terms: the scale that the rounding error of an FP32 evaluation in any
 * order is proportional to.
 * Derivation (Eq. 2 with T_k = prod_{j<k}(1 - alpha_j), w_k = alpha_k T_k):
 *   dC/drgb_k = w_k;
 *   dC/dalpha_k = rgb_k T_k - (sum_{j>k} rgb_j w_j + T_final bg) / (1 - alpha_k);
 *   alpha = o G unless clamped at 0.99 (then no gradient through o or G);
 *   dG/dmean2d = G Q d with d = p - mean2d; dG/da = -G dx^2/2, dG/db = -G dx dy,
 *   dG/dc = -G dy^2/2.
 * Each pixel's terms are computed independently (in parallel over pixels) and
 * then added into the outputs pixel by pixel in input order, so the sums are
 * the same, bit for bit, for any number of threads. */
typedef struct {
    int32_t idx, clamped;
    double g[9], a[9];   /* the pixel's terms of grad and g_abs for Gaussian idx */
} term_t;

/* the terms one pixel contributes, in compositing order; returns their count
 * (*out is malloc'ed, NULL when there are none) */
static int64_t pixel_adjoint_terms(int64_t n, const double* mean2d, const double* conic,
                                   const double* opacity, const double* rgb,
                                   const uint32_t* depth_key, const int32_t* visible, double px,
                                   double py, const double* bg, const double* g, cand_t* cand,
                                   double* Tk, term_t** out) {
    double mg;
    int64_t m = pixel_candidates(n, mean2d, conic, opacity, depth_key, visible, px, py, cand, &mg);
    double T = 1.0;
    int64_t used = 0;
    for (int64_t j = 0; j < m; ++j) {
        const double Tn = T * (1.0 - cand[j].alpha);
        if (Tn < T_MIN) break;
        Tk[j] = T;
        T = Tn;
        ++used;
    }
    *out = NULL;
    if (used == 0) return 0;
    term_t* t = (term_t*)calloc((size_t)used, sizeof(term_t));
    const double Tf = T;
    for (int64_t j = 0; j < used; ++j) {
        const int32_t i = cand[j].idx;
        const double al = cand[j].alpha;
        t[j].idx = i;
        t[j].clamped = cand[j].clamped;
        /* colour of everything behind j, including the background */
        double behind[3];
        for (int c = 0; c < 3; ++c) behind[c] = Tf * bg[c];
        for (int64_t h = j + 1; h < used; ++h) {
            const int32_t ih = cand[h].idx;
            for (int c = 0; c < 3; ++c) behind[c] += rgb[3 * ih + c] * cand[h].alpha * Tk[h];
        }
        /* dal: dL/dalpha; dal_abs: the sum of the magnitudes of its terms (the
         * scale of the rounding error of any evaluation of it) */
        double dal = 0.0, dal_abs = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double front = rgb[3 * i + c] * Tk[j], back = behind[c] / (1.0 - al);
            dal += g[c] * (front - back);
            dal_abs += fabs(g[c]) * (fabs(front) + fabs(back));
            const double dr = g[c] * al * Tk[j];
            t[j].g[6 + c] = dr;
            t[j].a[6 + c] = fabs(dr);
        }
        if (cand[j].clamped) continue;
        const double G = cand[j].G, o = opacity[i];
        const double dG = dal * o, dG_abs = dal_abs * o;
        t[j].g[5] = dal * G;
        t[j].a[5] = dal_abs * G;
        const double dx = px - mean2d[2 * i], dy = py - mean2d[2 * i + 1];
        const double a = conic[3 * i], b = conic[3 * i + 1], c = conic[3 * i + 2];
        t[j].g[0] = dG * G * (a * dx + b * dy);
        t[j].g[1] = dG * G * (b * dx + c * dy);
        t[j].a[0] = dG_abs * G * (fabs(a * dx) + fabs(b * dy));
        t[j].a[1] = dG_abs * G * (fabs(b * dx) + fabs(c * dy));
        t[j].g[2] = -0.5 * dG * G * dx * dx;
        t[j].g[3] = -dG * G * dx * dy;
        t[j].g[4] = -0.5 * dG * G * dy * dy;
        t[j].a[2] = 0.5 * dG_abs * G * dx * dx;
        t[j].a[3] = dG_abs * G * fabs(dx * dy);
        t[j].a[4] = 0.5 * dG_abs * G * dy * dy;
    }
    *out = t;
    return used;
}

void oracle_render_backward_pixels(int64_t n, const double* mean2d, const double* conic,
                                   const double* opacity, const double* rgb,
                                   const uint32_t* depth_key, const int32_t* visible,
                                   int64_t npix, const int32_t* pix, const double* bg,
                                   const double* dL_dC, double* grad, double* g_abs) {
    enum { BLOCK = 512 };
    term_t* terms[BLOCK];
    int64_t nterms[BLOCK];
    for (int64_t k0 = 0; k0 < npix; k0 += BLOCK) {
        const int64_t kb = npix - k0 < BLOCK ? npix - k0 : BLOCK;
#pragma omp parallel
        {
            cand_t* cand = (cand_t*)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
            double* Tk = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
            for (int64_t k = 0; k < kb; ++k) {
                const int64_t p = k0 + k;
                nterms[k] = pixel_adjoint_terms(n, mean2d, conic, opacity, rgb, depth_key, visible,
                                                pix[2 * p] + 0.5, pix[2 * p + 1] + 0.5, bg,
                                                dL_dC + 3 * p, cand, Tk, &terms[k]);
            }
            free(Tk);
            free(cand);
        }
        /* pixel order, then compositing order: the order a serial walk adds in */
        for (int64_t k = 0; k < kb; ++k) {
            for (int64_t j = 0; j < nterms[k]; ++j) {
                const term_t* t = &terms[k][j];
                const int64_t i = t->idx;
                for (int c = 0; c < 3; ++c) {
                    grad[9 * i + 6 + c] += t->g[6 + c];
                    g_abs[9 * i + 6 + c] += t->a[6 + c];
                }
                if (t->clamped) continue;
                grad[9 * i + 5] += t->g[5];
                g_abs[9 * i + 5] += t->a[5];
                for (int u = 0; u < 5; ++u) {
                    grad[9 * i + u] += t->g[u];
                    g_abs[9 * i + u] += t->a[u];
                }
            }
            free(terms[k]);
        }
    }
}

/* Thread count of the OpenMP regions above (the CPU-baseline timing runs the
 * oracle on one thread and on every core). */
void oracle_set_threads(int threads) { omp_set_num_threads(threads > 0 ? threads : 1); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Chain rule to the raw parameters                                           */
/* ------------------------------------------------------------------------ */
/* For Gaussians i in [0, n) with visible[i]: given g_proj (n x 9, layout as
 * above) accumulate raw-parameter gradients (summed into the outputs, so the
 * caller sums views by calling once per view):
 *   d_means[3][n], d_log_scales[3][n], d_quats[4][n], d_logits[n], d_sh[K][3][n].
 * Also the densification statistic of this view (Preliminary, last
 * paragraph; read as the mean over views of the per-view norm of the
 * position gradient in NDC units): accum[i] += ||(g_x W/2, g_y H/2)||,
 * denom[i] += 1 when visible.  Pass accum = NULL to skip. */
void oracle_project_backward(int64_t n, int deg, const float* means, const float* log_scales,
                             const float* quats, const float* logits, const float* sh,
                             const double* cam, int W, int H, double near_plane,
                             const int32_t* visible, const double* g_proj, double* d_means,
                             double* d_log_scales, double* d_quats, double* d_logits,
                             double* d_sh, double* accum, double* denom) {
    const double* Rw = cam;
    const double fx = cam[12], fy = cam[13];
    const int K = (deg + 1) * (deg + 1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (!visible[i]) continue;
        proj_t p;
        project_one(i, n, deg, means, log_scales, quats, logits, sh, cam, W, H, near_plane, &p);
        if (p.culled) continue;
        const double* g = g_proj + 9 * i;
        double gmu[3] = {0, 0, 0};
        /* opacity = sigmoid(logit) */
        d_logits[i] += g[5] * p.o * (1.0 - p.o);
        /* colour: rgb = max(0, sum_k Y_k f_k + 1/2) */
        double Y[16], dY[48];
        oracle_sh_basis(deg, p.dir, Y, dY);
        double gdir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ++ch) {
            if (p.rgb_pre[ch] < 0) continue;
            const double gr = g[6 + ch];
            for (int k = 0; k < K; ++k) {
                d_sh[((int64_t)k * 3 + ch) * n + i] += Y[k] * gr;
                const double f = sh[((int64_t)k * 3 + ch) * n + i];
                for (int a = 0; a < 3; ++a) gdir[a] += gr * f * dY[3 * k + a];
            }
        }
        /* dir = (mu - cc)/|mu - cc|: tangent projection / distance */
        double dd = p.dir[0] * gdir[0] + p.dir[1] * gdir[1] + p.dir[2] * gdir[2];
        for (int a = 0; a < 3; ++a) gmu[a] += (gdir[a] - p.dir[a] * dd) / p.dist;

        /* conic (a,b,c) -> Sigma' :  G_Sigma' = -Q G_Q Q, G_Q = [[ga, gb/2],[gb/2, gc]] */
        const double Q[4] = {p.conic[0], p.conic[1], p.conic[1], p.conic[2]};
        const double GQ[4] = {g[2], 0.5 * g[3], 0.5 * g[3], g[4]};
        double QG[4], GS2[4];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) QG[2 * a + b] = Q[2 * a] * GQ[b] + Q[2 * a + 1] * GQ[2 + b];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) GS2[2 * a + b] = -(QG[2 * a] * Q[b] + QG[2 * a + 1] * Q[2 + b]);
        /* Sigma' = T Sigma T^T + 0.3 I:  G_Sigma = T^T G_Sigma' T,  G_T = 2 G_Sigma' T Sigma */
        double GSig[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = 0;
                for (int u = 0; u < 2; ++u)
                    for (int w = 0; w < 2; ++w) v += p.T[3 * u + a] * GS2[2 * u + w] * p.T[3 * w + b];
                GSig[3 * a + b] = v;
            }
        double TSig[6], GT[6];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = 0;
                for (int k = 0; k < 3; ++k) v += p.T[3 * a + k] * p.Sigma[3 * k + b];
                TSig[3 * a + b] = v;
            }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) GT[3 * a + b] = 2.0 * (GS2[2 * a] * TSig[b] + GS2[2 * a + 1] * TSig[3 + b]);
        /* T = J W:  G_J = G_T W^T */
        double GJ[6];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = 0;
                for (int k = 0; k < 3; ++k) v += GT[3 * a + k] * Rw[3 * b + k];
                GJ[3 * a + b] = v;
            }
        /* J(t) with clamped x/z, y/z */
        const double tz = p.t[2];
        double gt[3] = {0, 0, 0};
        gt[2] += GJ[0] * (-fx / (tz * tz)) + GJ[4] * (-fy / (tz * tz));
        if (!p.clampx) {
            /* J02 = -fx tx / tz^2 */
            gt[0] += GJ[2] * (-fx / (tz * tz));
            gt[2] += GJ[2] * (2.0 * fx * p.t[0] / (tz * tz * tz));
        } else {
            gt[2] += GJ[2] * (fx * p.xt / (tz * tz));
        }
        if (!p.clampy) {
            gt[1] += GJ[5] * (-fy / (tz * tz));
            gt[2] += GJ[5] * (2.0 * fy * p.t[1] / (tz * tz * tz));
        } else {
            gt[2] += GJ[5] * (fy * p.yt / (tz * tz));
        }
        /* mean2d = (fx tx/tz + cx, fy ty/tz + cy) */
        gt[0] += g[0] * fx / tz;
        gt[1] += g[1] * fy / tz;
        gt[2] += -g[0] * fx * p.t[0] / (tz * tz) - g[1] * fy * p.t[1] / (tz * tz);
        /* t = W mu + t_w */
        for (int a = 0; a < 3; ++a) gmu[a] += Rw[a] * gt[0] + Rw[3 + a] * gt[1] + Rw[6 + a] * gt[2];
        /* Sigma = M M^T, M = R S:  G_M = 2 G_Sigma M */
        double M[9], GM[9], GR[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[3 * a + b] = p.R[3 * a + b] * p.s[b];
        mat3_mul(GSig, M, GM);
        for (int a = 0; a < 9; ++a) GM[a] *= 2.0;
        double gs[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                GR[3 * a + b] = GM[3 * a + b] * p.s[b];
                gs[b] += GM[3 * a + b] * p.R[3 * a + b];
            }
        double gqn[4];
        quat_to_rot_grad(p.qn, GR, gqn);
        double dq = 0;
        for (int a = 0; a < 4; ++a) dq += p.qn[a] * gqn[a];
        for (int a = 0; a < 4; ++a) d_quats[a * n + i] += (gqn[a] - p.qn[a] * dq) / p.qnorm;
        for (int a = 0; a < 3; ++a) d_log_scales[a * n + i] += gs[a] * p.s[a];
        for (int a = 0; a < 3; ++a) d_means[a * n + i] += gmu[a];
        if (accum) {
            const double gx = g[0] * 0.5 * W, gy = g[1] * 0.5 * H;
            accum[i] += sqrt(gx * gx + gy * gy);
            denom[i] += 1.0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                          */
/* ------------------------------------------------------------------------ */
/* Ten rounds of the Philox S-box on a 4x32 counter with a 2x32 key.  Each
 * round multiplies counter words 0 and 2 by the two round multipliers,
 * exchanges the halves and XORs in the key; the key is advanced by the two
 * Weyl increments between rounds. */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c0;
        const uint64_t p1 = (uint64_t)M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n1 = lo1;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        const uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Three standard normals for split child `child` of parent `parent` at
 * densification step `step`:  counter = (parent lo, parent hi, child, step),
 * key = (seed lo, seed hi);  u1 = ((x0 >> 8) + 1) 2^-24 in (0, 1],
 * u2 = (x1 >> 8) 2^-24, z0 = r cos(2 pi u2), z1 = r sin(2 pi u2) with
 * r = sqrt(-2 ln u1) (Box-Muller); z2 from (x2, x3) the same way, cosine branch.
 * words[4] receives the raw Philox output. */
void oracle_split_normals(uint64_t seed, uint64_t step, int64_t parent, int child, double z[3],
                          uint32_t words[4]) {
    const uint32_t ctr[4] = {(uint32_t)((uint64_t)parent & 0xffffffffu),
                             (uint32_t)((uint64_t)parent >> 32), (uint32_t)child, (uint32_t)step};
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    oracle_philox4x32_10(ctr, key, x);
    const double s24 = 1.0 / 16777216.0;
    const double u1 = ((x[0] >> 8) + 1) * s24, u2 = (x[1] >> 8) * s24;
    const double u3 = ((x[2] >> 8) + 1) * s24, u4 = (x[3] >> 8) * s24;
    const double r = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    z[0] = r * cos(2.0 * M_PI * u2);
    z[1] = r * sin(2.0 * M_PI * u2);
    z[2] = r2 * cos(2.0 * M_PI * u4);
    if (words)
        for (int a = 0; a < 4; ++a) words[a] = x[a];
}

/* Split children positions mu + R(q) (s * z) for a list of (parent, child)
 * pairs (FP64).  out[3k..3k+2]. */
void oracle_split_means(int64_t n, const float* means, const float* log_scales, const float* quats,
                        int64_t m, const int64_t* parent, const int32_t* child, uint64_t seed,
                        uint64_t step, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        const int64_t i = parent[k];
        double z[3];
        oracle_split_normals(seed, step, i, child[k], z, NULL);
        double q[4], R[9];
        double qn = 0;
        for (int a = 0; a < 4; ++a) {
            q[a] = quats[a * n + i];
            qn += q[a] * q[a];
        }
        qn = sqrt(qn);
        for (int a = 0; a < 4; ++a) q[a] /= qn;
        quat_to_rot(q, R);
        double v[3];
        for (int a = 0; a < 3; ++a) v[a] = exp((double)log_scales[a * n + i]) * z[a];
        for (int a = 0; a < 3; ++a)
            out[3 * k + a] = means[a * n + i] + R[3 * a] * v[0] + R[3 * a + 1] * v[1] + R[3 * a + 2] * v[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Densification statistic in the precision of its decision                  */
/* ------------------------------------------------------------------------ */
/* The split/clone masks compare the running statistic with a threshold, so
 * the statistic that feeds that decision is accumulated here in FP32 with a
 * fixed operation order (views in order; per view gx = g_x * (W/2),
 * gy = g_y * (H/2), norm = sqrt(fma(gx, gx, gy * gy)) correctly rounded,
 * accum += norm, denom += 1).  dmean2d is [V][2][n], visible [V][n]. */
void oracle_stats_f32(int64_t n, int32_t V, const float* dmean2d, const int32_t* visible,
                      const int32_t* wh, float* accum, float* denom) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float a = accum[i], d = denom[i];
        for (int32_t v = 0; v < V; ++v) {
            if (!visible[(int64_t)v * n + i]) continue;
            const float sx = (float)wh[2 * v] * 0.5f, sy = (float)wh[2 * v + 1] * 0.5f;
            const float gx = dmean2d[((int64_t)v * 2) * n + i] * sx;
            const float gy = dmean2d[((int64_t)v * 2 + 1) * n + i] * sy;
            const float nrm = sqrtf(fmaf(gx, gx, gy * gy));
            a = a + nrm;
            d = d + 1.0f;
        }
        accum[i] = a;
        denom[i] = d;
    }
}

/* Masks (Preliminary, last paragraph): avg = accum/denom (0 when denom = 0)
 * in FP32; a Gaussian is "hot" when avg >= tau_g and "large" when its largest
 * log-scale exceeds ln(rho E).  What a hot Gaussian becomes depends on mode:
 *   0  global phase of the global-to-local framework: large ones split, no clones
 *   1  the 3DGS rule: large ones split, the others clone
 *   2  split-only variant (Gaussian distribution comparison): every hot one splits
 *   3  clone-only variant: every hot one clones
 * prune = logit < logit(tau_o).  Thresholds are given in raw-parameter space
 * (log-scale and logit) so every decision is an exact FP32 comparison. */
void oracle_select(int64_t n, const float* accum, const float* denom, const float* log_scales,
                   const float* logits, float tau_g, float log_scale_thr, float logit_thr,
                   int mode, uint8_t* split, uint8_t* clone, uint8_t* prune) {
    for (int64_t i = 0; i < n; ++i) {
        const float avg = denom[i] > 0.0f ? accum[i] / denom[i] : 0.0f;
        float mx = log_scales[i];
        if (log_scales[n + i] > mx) mx = log_scales[n + i];
        if (log_scales[2 * n + i] > mx) mx = log_scales[2 * n + i];
        const int hot = avg >= tau_g;
        const int large = mx > log_scale_thr;
        int s = 0, c = 0;
        switch (mode) {
            case 0: s = hot && large; break;
            case 1: s = hot && large; c = hot && !large; break;
            case 2: s = hot; break;
            case 3: c = hot; break;
        }
        split[i] = (uint8_t)s;
        clone[i] = (uint8_t)c;
        prune[i] = (uint8_t)(logits[i] < logit_thr);
    }
}

/* Sigma = R(q/|q|) diag(exp(l))^2 R^T for one Gaussian (Eq. 1), row-major. */
void oracle_covariance3d(const double q[4], const double log_scale[3], double Sigma[9]) {
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double u[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
    double R[9], M[9], Mt[9];
    quat_to_rot(u, R);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[3 * a + b] = R[3 * a + b] * exp(log_scale[b]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Mt[3 * a + b] = M[3 * b + a];
    mat3_mul(M, Mt, Sigma);
}
