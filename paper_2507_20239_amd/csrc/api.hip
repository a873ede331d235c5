// Host side of the C ABI declared in gsmi.h: argument validation, the frame
// workspace layout, and the entry points that enqueue the kernels.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gs_internal.h"

static thread_local char g_err[512] = "no error";

gs_status gs_fail(gs_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

gs_status gs_check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return gs_fail(GS_ERR_HIP, "%s launch failed: %s", what, hipGetErrorString(e));
    return GS_OK;
}

namespace {

uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

struct Layout {
    uint64_t off[40];
    int count = 0;
    uint64_t total = 0;
    uint64_t add(uint64_t bytes) {
        const uint64_t o = total;
        off[count++] = o;
        total += align256(bytes > 0 ? bytes : 1);
        return o;
    }
};

gs_status check_views(int64_t n, int32_t V, const int32_t* widths, const int32_t* heights,
                      int64_t cap) {
    if (n < 0) return gs_fail(GS_ERR_INVALID, "n must be >= 0");
    if (V < 1 || V > GS_MAX_VIEWS) return gs_fail(GS_ERR_INVALID, "n_views must be in [1, %d]", GS_MAX_VIEWS);
    if (!widths || !heights) return gs_fail(GS_ERR_INVALID, "widths/heights are null");
    if ((int64_t)V * n >= ((int64_t)1 << 30)) return gs_fail(GS_ERR_INVALID, "n_views * n must be < 2^30");
    if (cap < 1 || cap >= ((int64_t)1 << 30)) return gs_fail(GS_ERR_INVALID, "max_instances must be in [1, 2^30)");
    int64_t tiles = 0;
    for (int v = 0; v < V; ++v) {
        if (widths[v] <= 0 || heights[v] <= 0 || widths[v] > 16384 || heights[v] > 16384)
            return gs_fail(GS_ERR_INVALID, "view %d: size %dx%d out of range", v, widths[v], heights[v]);
        tiles += (int64_t)((widths[v] + GS_TILE - 1) / GS_TILE) * ((heights[v] + GS_TILE - 1) / GS_TILE);
    }
    if (tiles >= ((int64_t)1 << 24)) return gs_fail(GS_ERR_INVALID, "too many tiles");
    return GS_OK;
}

void fill_views(gs_frame* f, const int32_t* widths, const int32_t* heights) {
    int32_t tb = 0;
    int64_t pb = 0;
    for (int v = 0; v < f->V; ++v) {
        gs_view_info& vi = f->views[v];
        vi.width = widths[v];
        vi.height = heights[v];
        vi.tiles_x = (widths[v] + GS_TILE - 1) / GS_TILE;
        vi.tiles_y = (heights[v] + GS_TILE - 1) / GS_TILE;
        vi.tile_base = tb;
        vi.pad = 0;
        vi.pix_base = pb;
        tb += vi.tiles_x * vi.tiles_y;
        pb += (int64_t)widths[v] * heights[v];
    }
    f->T = tb;
    f->P = pb;
    // tile keys hold 0..T, T being the never-taken 'no tile' value of the emission
    int bits = 1;
    while (((int64_t)1 << bits) <= (int64_t)tb) ++bits;
    f->tile_bits = bits;
}

Layout layout_for(gs_frame* f) {
    const uint64_t E = (uint64_t)f->E, cap = (uint64_t)f->cap, T = (uint64_t)f->T, P = (uint64_t)f->P;
    uint64_t sort_bytes = gs_radix_scratch_bytes(f->cap, f->tile_bits);
    const uint64_t st = gs_radix_scratch_bytes(f->T, 24);
    if (st > sort_bytes) sort_bytes = st;
    const uint64_t sd = gs_radix_scratch_bytes(f->E, 32);
    if (sd > sort_bytes) sort_bytes = sd;
    Layout L;
    L.add(4 * E);        // 0 depth_key
    L.add(4 * E);        // 1 tiles_touched
    L.add(8 * E);        // 2 rect
    L.add(48 * E);       // 3 splat
    L.add(4 * E);        // 4 visible
    L.add(4 * E);        // 5 inst_off
    L.add(4 * cap);      // 6 ikeys0
    L.add(4 * cap);      // 7 ikeys1
    L.add(4 * cap);      // 8 ivals0
    L.add(4 * cap);      // 9 ivals1
    L.add(8 * T);        // 10 ranges
    L.add(4 * T);        // 11 tkeys0
    L.add(4 * T);        // 12 tkeys1
    L.add(4 * T);        // 13 tvals0
    L.add(4 * T);        // 14 tvals1
    L.add(4 * P);        // 15 T_final
    L.add(4 * P);        // 16 n_contrib
    L.add(36 * E);       // 17 splat_grad
    L.add(64);           // 18 counters
    L.add(sort_bytes);   // 19 sort scratch
    L.add(16 * (GS_SCAN_PARTS + 8));  // 20 scan_part
    L.add(sizeof(gs_view_info) * GS_MAX_VIEWS);  // 21 views
    L.add(4 * P);        // 22 n_comp
    L.add(4 * (cap / 256 + 2));  // 23 chunk_start
    L.add(4 * E);        // 24 dkeys0
    L.add(4 * E);        // 25 dkeys1
    L.add(4 * E);        // 26 dvals1
    return L;
}

gs_status check_frame(const gs_frame* f) {
    if (!f) return gs_fail(GS_ERR_INVALID, "frame is null");
    return GS_OK;
}

gs_status check_gaussians(const gs_frame* f, const gs_gaussians* g) {
    if (!g) return gs_fail(GS_ERR_INVALID, "gaussians is null");
    if (g->n != f->n) return gs_fail(GS_ERR_INVALID, "gaussians n=%lld but the frame was made for n=%lld",
                                     (long long)g->n, (long long)f->n);
    if (g->sh_degree < 0 || g->sh_degree > 3) return gs_fail(GS_ERR_INVALID, "sh_degree must be in [0, 3]");
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
        return gs_fail(GS_ERR_INVALID, "a Gaussian parameter pointer is null");
    return GS_OK;
}

gs_status check_opts(const gs_raster_opts* o) {
    if (!o) return gs_fail(GS_ERR_INVALID, "opts is null");
    if (o->raster_batch != 0 && o->raster_batch != 64 && o->raster_batch != 128 && o->raster_batch != 256)
        return gs_fail(GS_ERR_INVALID, "raster_batch must be 0, 64, 128 or 256");
    if (o->persistent_blocks < 0 || o->persistent_blocks > 65536)
        return gs_fail(GS_ERR_INVALID, "persistent_blocks must be in [0, 65536]");
    if (o->flags & ~(GS_RASTER_COUNT_COMPOSITED | GS_RASTER_FOOTPRINT_3SIGMA | GS_RASTER_DEPTH_PRESORT |
                     GS_RASTER_BALANCED_DIGITS | GS_RASTER_GRAD_RENDERED_ONLY |
                     GS_RASTER_LANE_PIXELS | GS_RASTER_LANE_QUADS))
        return gs_fail(GS_ERR_INVALID, "unknown bits in raster flags");
    if ((o->flags & GS_RASTER_LANE_PIXELS) && (o->flags & GS_RASTER_LANE_QUADS))
        return gs_fail(GS_ERR_INVALID, "GS_RASTER_LANE_PIXELS and GS_RASTER_LANE_QUADS exclude each other");
    if ((o->flags & GS_RASTER_LANE_PIXELS) && o->persistent_blocks > 0)
        return gs_fail(GS_ERR_INVALID, "one pixel per lane runs on the plain grid (persistent_blocks = 0)");
    if (!(o->near_plane > 0.f)) return gs_fail(GS_ERR_INVALID, "near_plane must be > 0");
    return GS_OK;
}

}  // namespace

struct gs_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

const char* gs_last_error(void) { return g_err; }
const char* gs_version(void) { return "gsmi 0.1 (gfx950)"; }

gs_status gs_frame_workspace_size(int64_t n, int32_t n_views, const int32_t* widths,
                                  const int32_t* heights, int64_t max_instances, uint64_t* bytes) {
    GS_TRY(check_views(n, n_views, widths, heights, max_instances));
    if (!bytes) return gs_fail(GS_ERR_INVALID, "bytes is null");
    gs_frame f;
    memset(&f, 0, sizeof f);
    f.n = n;
    f.V = n_views;
    f.E = n * n_views;
    f.cap = max_instances;
    fill_views(&f, widths, heights);
    *bytes = layout_for(&f).total;
    return GS_OK;
}

gs_status gs_frame_create(int64_t n, int32_t n_views, const int32_t* widths,
                          const int32_t* heights, int64_t max_instances, void* workspace,
                          uint64_t workspace_bytes, gs_frame** out) {
    GS_TRY(check_views(n, n_views, widths, heights, max_instances));
    if (!out || !workspace) return gs_fail(GS_ERR_INVALID, "null pointer");
    if (((uintptr_t)workspace & 255) != 0) return gs_fail(GS_ERR_INVALID, "workspace must be 256-byte aligned");
    gs_frame* f = (gs_frame*)calloc(1, sizeof(gs_frame));
    if (!f) return gs_fail(GS_ERR_INVALID, "out of host memory");
    f->n = n;
    f->V = n_views;
    f->E = n * n_views;
    f->cap = max_instances;
    fill_views(f, widths, heights);
    Layout L = layout_for(f);
    if (workspace_bytes < L.total) {
        free(f);
        return gs_fail(GS_ERR_INVALID, "workspace too small (%llu < %llu)",
                       (unsigned long long)workspace_bytes, (unsigned long long)L.total);
    }
    char* b = (char*)workspace;
    f->depth_key = (u32*)(b + L.off[0]);
    f->tiles_touched = (u32*)(b + L.off[1]);
    f->rect = (uint2*)(b + L.off[2]);
    f->splat = (float4*)(b + L.off[3]);
    f->visible = (u32*)(b + L.off[4]);
    f->inst_off = (u32*)(b + L.off[5]);
    f->ikeys[0] = (u32*)(b + L.off[6]);
    f->ikeys[1] = (u32*)(b + L.off[7]);
    f->ivals[0] = (u32*)(b + L.off[8]);
    f->ivals[1] = (u32*)(b + L.off[9]);
    f->ranges = (uint2*)(b + L.off[10]);
    f->tkeys[0] = (u32*)(b + L.off[11]);
    f->tkeys[1] = (u32*)(b + L.off[12]);
    f->tvals[0] = (u32*)(b + L.off[13]);
    f->tvals[1] = (u32*)(b + L.off[14]);
    f->T_final = (float*)(b + L.off[15]);
    f->n_contrib = (u32*)(b + L.off[16]);
    f->splat_grad = (float*)(b + L.off[17]);
    f->counters = (u32*)(b + L.off[18]);
    f->sort_scratch = (void*)(b + L.off[19]);
    f->scan_part = (u32*)(b + L.off[20]);
    f->d_views = (gs_view_info*)(b + L.off[21]);
    f->n_comp = (u32*)(b + L.off[22]);
    f->chunk_start = (u32*)(b + L.off[23]);
    f->dkeys[0] = (u32*)(b + L.off[24]);
    f->dkeys[1] = (u32*)(b + L.off[25]);
    f->dvals1 = (u32*)(b + L.off[26]);
    // the slot holding the sorted instances depends only on the pass count; the
    // heavy-first order exists only after a binning that built it
    f->isorted = (((f->tile_bits + 7) / 8) & 1);
    f->tsorted = 0;
    f->heavy_built = false;
    hipError_t e = hipMemcpy(f->d_views, f->views, sizeof(gs_view_info) * n_views, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(f->counters, 0, 64);
    if (e != hipSuccess) {
        free(f);
        return gs_fail(GS_ERR_HIP, "frame upload failed: %s", hipGetErrorString(e));
    }
    *out = f;
    return GS_OK;
}

gs_status gs_frame_destroy(gs_frame* frame) {
    free(frame);
    return GS_OK;
}

gs_status gs_frame_buffer(const gs_frame* f, int32_t which, void** ptr, int64_t* count) {
    GS_TRY(check_frame(f));
    if (!ptr || !count) return gs_fail(GS_ERR_INVALID, "null pointer");
    switch (which) {
        case GS_BUF_DEPTH_KEY: *ptr = f->depth_key; *count = f->E; break;
        case GS_BUF_TILES_TOUCHED: *ptr = f->tiles_touched; *count = f->E; break;
        case GS_BUF_RECT: *ptr = f->rect; *count = 2 * f->E; break;
        case GS_BUF_SPLAT: *ptr = f->splat; *count = 12 * f->E; break;
        case GS_BUF_VISIBLE: *ptr = f->visible; *count = f->E; break;
        case GS_BUF_INST_TILE: *ptr = f->ikeys[f->isorted]; *count = f->cap; break;
        case GS_BUF_INST_ENTRY: *ptr = f->ivals[f->isorted]; *count = f->cap; break;
        case GS_BUF_RANGES: *ptr = f->ranges; *count = 2 * (int64_t)f->T; break;
        case GS_BUF_T_FINAL: *ptr = f->T_final; *count = f->P; break;
        case GS_BUF_N_CONTRIB: *ptr = f->n_contrib; *count = f->P; break;
        case GS_BUF_SPLAT_GRAD: *ptr = f->splat_grad; *count = 9 * f->E; break;
        case GS_BUF_COUNTERS: *ptr = f->counters; *count = 16; break;
        case GS_BUF_N_COMPOSITED: *ptr = f->n_comp; *count = f->P; break;
        default: return gs_fail(GS_ERR_INVALID, "unknown buffer id %d", which);
    }
    return GS_OK;
}

gs_status gs_frame_status(gs_frame* f, void* stream, int64_t* n_visible, int64_t* n_instances,
                          int32_t* overflow) {
    GS_TRY(check_frame(f));
    u32 h[8];
    GS_HIP(hipStreamSynchronize((hipStream_t)stream));
    GS_HIP(hipMemcpy(h, f->counters, sizeof h, hipMemcpyDeviceToHost));
    if (n_visible) *n_visible = h[0];
    if (n_instances) *n_instances = h[1];
    if (overflow) *overflow = (int32_t)h[2];
    return h[2] ? gs_fail(GS_ERR_CAPACITY, "instance capacity %lld exceeded (%u needed)",
                          (long long)f->cap, h[1])
                : GS_OK;
}

gs_status gs_project(gs_frame* f, const gs_gaussians* g, const gs_camera* cameras,
                     const gs_raster_opts* opts, void* stream) {
    GS_TRY(check_frame(f));
    GS_TRY(check_gaussians(f, g));
    GS_TRY(check_opts(opts));
    if (!cameras) return gs_fail(GS_ERR_INVALID, "cameras is null");
    return gs_launch_project(f, g, cameras, opts->near_plane,
                             (opts->flags & GS_RASTER_FOOTPRINT_3SIGMA) != 0, (hipStream_t)stream);
}

gs_status gs_bin(gs_frame* f, const gs_raster_opts* opts, void* stream) {
    GS_TRY(check_frame(f));
    GS_TRY(check_opts(opts));
    return gs_launch_bin(f, (hipStream_t)stream, opts->persistent_blocks > 0,
                         (opts->flags & GS_RASTER_DEPTH_PRESORT) != 0,
                         (opts->flags & GS_RASTER_BALANCED_DIGITS) != 0);
}

gs_status gs_composite(gs_frame* f, const gs_raster_opts* opts, float* images, void* stream) {
    GS_TRY(check_frame(f));
    GS_TRY(check_opts(opts));
    if (!images) return gs_fail(GS_ERR_INVALID, "images is null");
    if (opts->persistent_blocks > 0 && !f->heavy_built)
        return gs_fail(GS_ERR_INVALID,
                       "persistent_blocks > 0 needs the heavy-first tile order, which the last "
                       "binning did not build (it ran with persistent_blocks = 0)");
    return gs_launch_raster_fwd(f, opts, images, nullptr, 0.f, nullptr, nullptr,
                                (hipStream_t)stream);
}

gs_status gs_composite_l1(gs_frame* f, const gs_raster_opts* opts, float* images,
                          const float* targets, float l1_scale, float* loss, float* dL_dimages,
                          void* stream) {
    GS_TRY(check_frame(f));
    GS_TRY(check_opts(opts));
    if (!images || !targets || !loss || !dL_dimages) return gs_fail(GS_ERR_INVALID, "null pointer");
    if (opts->persistent_blocks > 0 && !f->heavy_built)
        return gs_fail(GS_ERR_INVALID,
                       "persistent_blocks > 0 needs the heavy-first tile order, which the last "
                       "binning did not build (it ran with persistent_blocks = 0)");
    return gs_launch_raster_fwd(f, opts, images, targets, l1_scale, loss, dL_dimages,
                                (hipStream_t)stream);
}

gs_status gs_render(gs_frame* f, const gs_raster_opts* opts, float* images, void* stream) {
    GS_TRY(check_frame(f));
    GS_TRY(check_opts(opts));
    if (!images) return gs_fail(GS_ERR_INVALID, "images is null");
    GS_TRY(gs_bin(f, opts, stream));
    return gs_composite(f, opts, images, stream);
}

gs_status gs_render_backward(gs_frame* f, const gs_raster_opts* opts, const float* dL_dimages,
                             void* stream) {
    GS_TRY(check_frame(f));
    GS_TRY(check_opts(opts));
    if (!dL_dimages) return gs_fail(GS_ERR_INVALID, "dL_dimages is null");
    if (opts->persistent_blocks > 0 && !f->heavy_built)
        return gs_fail(GS_ERR_INVALID,
                       "persistent_blocks > 0 needs the heavy-first tile order, which the last "
                       "gs_render did not build (it ran with persistent_blocks = 0)");
    return gs_launch_raster_bwd(f, opts, dL_dimages, (hipStream_t)stream);
}

gs_status gs_project_backward(gs_frame* f, const gs_gaussians* g, const gs_camera* cameras,
                              const gs_raster_opts* opts, const gs_gaussian_grads* grads,
                              float* accum, float* denom, void* stream) {
    GS_TRY(check_frame(f));
    GS_TRY(check_gaussians(f, g));
    GS_TRY(check_opts(opts));
    if (!cameras || !grads) return gs_fail(GS_ERR_INVALID, "null pointer");
    if (f->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits || !grads->sh))
        return gs_fail(GS_ERR_INVALID, "a gradient pointer is null");
    if ((accum == nullptr) != (denom == nullptr))
        return gs_fail(GS_ERR_INVALID, "accum and denom must both be set or both be null");
    return gs_launch_project_bwd(f, g, cameras, opts->near_plane, grads, accum, denom,
                                 (opts->flags & GS_RASTER_GRAD_RENDERED_ONLY) != 0, nullptr,
                                 (hipStream_t)stream);
}

gs_status gs_project_backward_adam(gs_frame* f, const gs_gaussians* g, const gs_camera* cameras,
                                   const gs_raster_opts* opts, const gs_gaussian_grads* grads,
                                   float* accum, float* denom, const gs_fused_adam* adam,
                                   void* stream) {
    GS_TRY(check_frame(f));
    GS_TRY(check_gaussians(f, g));
    GS_TRY(check_opts(opts));
    if (!cameras || !grads || !adam) return gs_fail(GS_ERR_INVALID, "null pointer");
    if ((accum == nullptr) != (denom == nullptr))
        return gs_fail(GS_ERR_INVALID, "accum and denom must both be set or both be null");
    const float* own[5] = {g->means, g->log_scales, g->quats, g->opacity_logits, g->sh};
    float* const grad[5] = {grads->means, grads->log_scales, grads->quats, grads->opacity_logits,
                            grads->sh};
    for (int k = 0; k < 5; ++k) {
        if (f->n == 0) break;
        if (!adam->param[k]) {
            if (!grad[k]) return gs_fail(GS_ERR_INVALID, "gradient %d is null and not fused", k);
            continue;
        }
        if (adam->param[k] != own[k])
            return gs_fail(GS_ERR_INVALID, "adam param %d must be the Gaussians' array (updated in place)", k);
        if (!adam->m[k] || !adam->v[k])
            return gs_fail(GS_ERR_INVALID, "adam param %d: null moment", k);
    }
    if (!(adam->beta1 >= 0.f && adam->beta1 < 1.f && adam->beta2 >= 0.f && adam->beta2 < 1.f &&
          adam->eps > 0.f))
        return gs_fail(GS_ERR_INVALID, "adam: need 0 <= beta < 1 and eps > 0");
    if (!adam->counter && adam->step < 1) return gs_fail(GS_ERR_INVALID, "adam: step counts from 1");
    if (adam->counter && ((uintptr_t)adam->counter & 7) != 0)
        return gs_fail(GS_ERR_INVALID, "adam: counter must be 8-byte aligned");
    return gs_launch_project_bwd(f, g, cameras, opts->near_plane, grads, accum, denom,
                                 (opts->flags & GS_RASTER_GRAD_RENDERED_ONLY) != 0, adam,
                                 (hipStream_t)stream);
}

gs_status gs_sort_workspace_size(int64_t n, uint64_t* bytes) {
    if (n < 0 || n >= ((int64_t)1 << 30) || !bytes) return gs_fail(GS_ERR_INVALID, "bad argument");
    *bytes = 2 * align256(4 * (uint64_t)(n > 0 ? n : 1)) + align256(gs_radix_scratch_bytes(n, 32));
    return GS_OK;
}

gs_status gs_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int32_t key_bits,
                        void* workspace, uint64_t workspace_bytes, void* stream) {
    if (key_bits < 1 || key_bits > 32) return gs_fail(GS_ERR_INVALID, "key_bits must be in [1, 32]");
    uint64_t need;
    GS_TRY(gs_sort_workspace_size(n, &need));
    if (n == 0) return GS_OK;
    if (!keys || !vals || !workspace) return gs_fail(GS_ERR_INVALID, "null pointer");
    if (workspace_bytes < need) return gs_fail(GS_ERR_INVALID, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    char* b = (char*)workspace;
    const uint64_t nb = align256(4 * (uint64_t)n);
    u32* k[2] = {keys, (u32*)b};
    u32* v[2] = {vals, (u32*)(b + nb)};
    void* scratch = (void*)(b + 2 * nb);
    int slot = 0;
    GS_TRY(gs_radix_sort(k, v, nullptr, (u32)n, n, key_bits, scratch, &slot, s));
    if (slot == 1) {
        GS_HIP(hipMemcpyAsync(keys, k[1], 4 * n, hipMemcpyDeviceToDevice, s));
        GS_HIP(hipMemcpyAsync(vals, v[1], 4 * n, hipMemcpyDeviceToDevice, s));
    }
    return GS_OK;
}

gs_status gs_step_graph_create(gs_frame* f, const gs_gaussians* g, const gs_camera* cameras,
                               const gs_raster_opts* opts, float* images, const float* targets,
                               float l1_scale, float* loss, float* dL_dimages,
                               const gs_gaussian_grads* grads, float* accum, float* denom,
                               void* stream, gs_graph** out) {
    GS_TRY(check_frame(f));
    GS_TRY(check_gaussians(f, g));
    GS_TRY(check_opts(opts));
    if (!cameras || !images || !targets || !loss || !dL_dimages || !grads || !out)
        return gs_fail(GS_ERR_INVALID, "null pointer");
    hipStream_t cs;
    GS_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    gs_status st = GS_OK;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return gs_fail(GS_ERR_HIP, "begin capture: %s", hipGetErrorString(e));
    }
    const int64_t numel = 3 * f->P;
    st = gs_project(f, g, cameras, opts, cs);
    if (st == GS_OK) st = gs_fill_u32((u32*)loss, 0u, 1, cs);
    if (st == GS_OK) st = gs_bin(f, opts, cs);
    if (st == GS_OK) st = gs_composite_l1(f, opts, images, targets, l1_scale, loss, dL_dimages, cs);
    if (st == GS_OK) st = gs_render_backward(f, opts, dL_dimages, cs);
    if (st == GS_OK) st = gs_project_backward(f, g, cameras, opts, grads, accum, denom, cs);
    e = hipStreamEndCapture(cs, &graph);
    if (st == GS_OK && e != hipSuccess) st = gs_fail(GS_ERR_HIP, "end capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    if (st == GS_OK) {
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = gs_fail(GS_ERR_HIP, "instantiate: %s", hipGetErrorString(e));
    }
    (void)hipStreamDestroy(cs);
    if (st != GS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    gs_graph* gr = (gs_graph*)calloc(1, sizeof(gs_graph));
    gr->graph = graph;
    gr->exec = exec;
    *out = gr;
    (void)stream;
    return GS_OK;
}

gs_status gs_graph_launch(gs_graph* graph, void* stream) {
    if (!graph) return gs_fail(GS_ERR_INVALID, "graph is null");
    GS_HIP(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return GS_OK;
}

gs_status gs_graph_destroy(gs_graph* graph) {
    if (!graph) return GS_OK;
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    free(graph);
    return GS_OK;
}

}  // extern "C"
