// Sparse Adam over the Gaussians rendered in the current step.
//
// The optimiser step that follows the projection adjoint in the accelerated
// 3DGS training the paper builds on (Experiments, implementation details and
// the footnote on its baseline): a Gaussian that no view rendered has a zero
// gradient and keeps its parameters and both moments untouched; every
// rendered Gaussian takes a standard Adam step with bias correction by the
// global step count t:
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
// One thread per Gaussian walks every row of every parameter array
// (structure of arrays: consecutive threads touch consecutive floats of a
// row), four rows at a time with all loads issued before the stores.  Every
// thread stores its parameter and moments back, a Gaussian outside the update
// storing the values it read: rendered Gaussians are scattered over the index
// range, so each cache line holds some of them anyway, and whole-line stores
// run faster than partial ones.  HBM-bound: 16 B read and 12 B written per
// float of every Gaussian.
#include "gs_internal.h"

namespace {

constexpr int ADAM_MAX_PARAMS = 8;

struct AdamTable {
    gs_adam_param p[ADAM_MAX_PARAMS];
    int count;
};

// The step count of a counted call: one thread advances the device counter
// and writes the two bias-correction factors next to it, as the host computes
// them for an uncounted call (FP64, rounded once).
__global__ void adam_count_kernel(gs_adam_counter* c, float b1, float b2) {
    if (threadIdx.x != 0) return;
    const int64_t t = c->step + 1;
    c->step = t;
    c->c1 = adam_bias_factor(b1, t);
    c->c2 = adam_bias_factor(b2, t);
}

__global__ void __launch_bounds__(GS_BLOCK) adam_kernel(AdamTable t, int64_t n,
                                                        const u32* __restrict__ tiles_touched,
                                                        int n_views, float b1, float b2,
                                                        float eps, float c1, float c2,
                                                        const gs_adam_counter* counter) {
    const int64_t i = (int64_t)blockIdx.x * GS_BLOCK + threadIdx.x;
    if (i >= n) return;
    if (counter) {
        c1 = counter->c1;
        c2 = counter->c2;
    }
    bool upd = true;
    if (tiles_touched) {
        u32 any = 0;
        for (int v = 0; v < n_views; ++v) any |= tiles_touched[(int64_t)v * n + i];
        upd = any != 0;
        // a wave with no rendered Gaussian leaves its rows as they are without
        // touching them (whole waves of them, when the Gaussians are in spatial order)
        if (__ballot(upd) == 0) return;
    }
    for (int a = 0; a < t.count; ++a) {
        const gs_adam_param q = t.p[a];
        int r = 0;
        for (; r + 4 <= q.rows; r += 4) {
            float m[4], v[4], p[4], g[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t k = (int64_t)(r + j) * n + i;
                m[j] = q.m[k];
                v[j] = q.v[k];
                p[j] = q.param[k];
                g[j] = upd ? q.grad[k] : 0.f;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t k = (int64_t)(r + j) * n + i;
                adam_element(upd, g[j], m[j], v[j], p[j], q.lr, b1, b2, eps, c1, c2);
                q.m[k] = m[j];
                q.v[k] = v[j];
                q.param[k] = p[j];
            }
        }
        for (; r < q.rows; ++r) {
            const int64_t k = (int64_t)r * n + i;
            float m = q.m[k], v = q.v[k], p = q.param[k];
            adam_element(upd, upd ? q.grad[k] : 0.f, m, v, p, q.lr, b1, b2, eps, c1, c2);
            q.m[k] = m;
            q.v[k] = v;
            q.param[k] = p;
        }
    }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + GS_BLOCK - 1) / GS_BLOCK); }

}  // namespace

namespace {

gs_status adam_launch(const gs_adam_param* params, int32_t n_params, int64_t n,
                      const uint32_t* tiles_touched, int32_t n_views, float beta1, float beta2,
                      float eps, int64_t step, gs_adam_counter* counter, hipStream_t s) {
    if (n < 0 || n_params < 0 || n_params > ADAM_MAX_PARAMS)
        return gs_fail(GS_ERR_INVALID, "n_params must be in [0, %d] and n >= 0", ADAM_MAX_PARAMS);
    if (!counter && step < 1) return gs_fail(GS_ERR_INVALID, "step counts from 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
        return gs_fail(GS_ERR_INVALID, "need 0 <= beta < 1 and eps > 0");
    if (tiles_touched && (n_views < 1 || n_views > GS_MAX_VIEWS))
        return gs_fail(GS_ERR_INVALID, "n_views must be in [1, %d]", GS_MAX_VIEWS);
    const bool work = n > 0 && n_params > 0;
    AdamTable t;
    t.count = n_params;
    if (work) {
        if (!params) return gs_fail(GS_ERR_INVALID, "params is null");
        for (int a = 0; a < n_params; ++a) {
            const gs_adam_param& q = params[a];
            if (!q.param || !q.grad || !q.m || !q.v || q.rows <= 0)
                return gs_fail(GS_ERR_INVALID, "parameter %d: null pointer or rows <= 0", a);
            t.p[a] = q;
        }
    }
    // a counted call advances its counter even when there is nothing to update,
    // so the count always equals the number of calls
    if (counter) {
        adam_count_kernel<<<1, 64, 0, s>>>(counter, beta1, beta2);
        GS_TRY(gs_check_launch("adam_count"));
    }
    if (!work) return GS_OK;
    float c1 = 1.f, c2 = 1.f;
    if (!counter) {
        c1 = adam_bias_factor(beta1, step);
        c2 = adam_bias_factor(beta2, step);
    }
    adam_kernel<<<blocks_for(n), GS_BLOCK, 0, s>>>(t, n, tiles_touched, n_views, beta1, beta2, eps,
                                                   c1, c2, counter);
    return gs_check_launch("adam_step");
}

}  // namespace

extern "C" gs_status gs_adam_step(const gs_adam_param* params, int32_t n_params, int64_t n,
                                  const uint32_t* tiles_touched, int32_t n_views, float beta1,
                                  float beta2, float eps, int64_t step, void* stream) {
    return adam_launch(params, n_params, n, tiles_touched, n_views, beta1, beta2, eps, step,
                       nullptr, (hipStream_t)stream);
}

extern "C" gs_status gs_adam_step_counted(const gs_adam_param* params, int32_t n_params, int64_t n,
                                          const uint32_t* tiles_touched, int32_t n_views,
                                          float beta1, float beta2, float eps,
                                          gs_adam_counter* counter, void* stream) {
    if (!counter) return gs_fail(GS_ERR_INVALID, "counter is null");
    if (((uintptr_t)counter & 7) != 0) return gs_fail(GS_ERR_INVALID, "counter must be 8-byte aligned");
    return adam_launch(params, n_params, n, tiles_touched, n_views, beta1, beta2, eps, 0, counter,
                       (hipStream_t)stream);
}
