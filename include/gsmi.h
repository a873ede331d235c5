/*
 * gsmi.h -- C ABI of the MI355X (gfx950) Gaussian-splatting hot path.
 *
 * Implements, as hand-written HIP kernels, the differentiable tile rasterizer
 * and the densification step of 3D Gaussian Splatting training as scheduled
 * in "Decomposing Densification in Gaussian Splatting for Faster 3D Scene
 * Reconstruction" (arXiv 2507.20239):
 *   - projection of anisotropic Gaussians (Eq. 1; Sigma = R S S^T R^T and
 *     Sigma' = J W Sigma W^T J^T, Preliminary) with spherical-harmonic colour;
 *   - depth-ordered front-to-back alpha compositing per 16x16 tile (Eq. 2)
 *     and its adjoint;
 *   - the densification statistic (norm of the view-space position gradient)
 *     and the split / clone / prune rule (Preliminary, last paragraph),
 *     including the clone suppression of the global phase (Methodology,
 *     Global-to-local framework);
 *   - the adaptive opacity threshold (Methodology, Adaptive Opacity Pruning).
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers unless the comment says "host".
 *     The caller owns every buffer it passes; the library never frees or
 *     keeps caller pointers after the call returns (a captured step graph,
 *     gs_step_graph_*, is the one exception and says so).
 *   - `stream` is a hipStream_t passed as void*; all work is enqueued on it
 *     asynchronously.  Entry points that must read a device value on the host
 *     say "synchronises".
 *   - Every call returns a gs_status.  Argument validation happens on the
 *     host before any launch; on error nothing is enqueued and
 *     gs_last_error() returns a description (thread-local).
 *   - Gaussian parameters are structure-of-arrays FP32 with the Gaussian
 *     index fastest: means[3][n], log_scales[3][n], quats[4][n] (w, x, y, z,
 *     any norm), opacity_logits[n], sh[K][3][n] with K = (sh_degree+1)^2,
 *     real spherical harmonics with the Condon-Shortley phase,
 *     colour = max(0, sum_k Y_k f_k + 1/2).
 *   - Cameras are world->camera rigid transforms in OpenCV axes (x right,
 *     y down, z forward); pixel (px, py) is sampled at (px+0.5, py+0.5).
 *   - Images are planar FP32 [3][H][W]; a frame with several views stores
 *     them one after the other in view order.
 *   - Rendering constants: alpha = min(0.99, o G); Gaussians with
 *     alpha < 1/255 are skipped at that pixel; a pixel stops before
 *     compositing a Gaussian that would take its transmittance below 1e-4;
 *     Sigma' gets +0.3 px^2 on its diagonal; x/z and y/z are clamped to
 *     +-1.3 tan(half field of view) inside J.
 */
#ifndef GSMI_H
#define GSMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID = 1,     /* bad argument; nothing was enqueued */
    GS_ERR_CAPACITY = 2,    /* a device-side capacity was exceeded (see gs_frame_status) */
    GS_ERR_HIP = 3,         /* a HIP runtime call failed */
    GS_ERR_UNSUPPORTED = 4  /* valid but not supported by the library */
} gs_status;

/* Text of the last non-OK status on the calling thread (never NULL). */
const char* gs_last_error(void);
/* Library version string. */
const char* gs_version(void);

#define GS_MAX_VIEWS 32
#define GS_TILE 16

/* One camera (72 bytes).  R: world->camera rotation, row-major; t: translation
 * (x_cam = R x_world + t); fx, fy, cx, cy: pinhole intrinsics in pixels for the
 * resolution being rendered (a coarse level 1/r divides all four by r);
 * width, height: image size in pixels.  Passed to kernels as a device array. */
typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
} gs_camera;

/* Gaussian parameters (device, FP32 SoA as described above). */
typedef struct {
    const float* means;          /* [3][n] */
    const float* log_scales;     /* [3][n] */
    const float* quats;          /* [4][n] */
    const float* opacity_logits; /* [n]    */
    const float* sh;             /* [K][3][n] */
    int64_t n;
    int32_t sh_degree;           /* 0..3 */
    int32_t reserved;
} gs_gaussians;

/* Gradients w.r.t. the raw parameters (device, same layouts; overwritten). */
typedef struct {
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* sh;
} gs_gaussian_grads;

/* Rasterisation options. */
typedef struct {
    float bg[3];                 /* background colour composited behind every pixel */
    float near_plane;            /* Gaussians with camera depth <= near are culled (default 0.2) */
    int32_t raster_batch;        /* Gaussians staged in LDS per batch: 64, 128 or 256; 0 = 64 */
    int32_t persistent_blocks;   /* 0: one wave64 workgroup per (view, tile);  > 0: a persistent
                                    grid of this many wave64 workgroups takes (view, tile) items
                                    from a queue, heaviest tile lists first */
    int32_t flags;               /* GS_RASTER_* bits */
    int32_t reserved;
} gs_raster_opts;

/* gs_raster_opts.flags: gs_render also counts, per pixel, the splats it
 * composited into GS_BUF_N_COMPOSITED (a diagnostic; without the flag that
 * buffer is left as it was). */
#define GS_RASTER_COUNT_COMPOSITED 1
/* gs_raster_opts.flags: gs_project bins every Gaussian in front of the camera
 * to the tiles whose 16x16 squares meet its 3-sigma square [u - r, u + r] x
 * [v - r, v + r], r = ceil(3 sqrt(largest eigenvalue of Sigma')) pixels,
 * whatever its opacity: the footprint of the original 3DGS rasterizer.  A
 * pixel then sees only the splats binned to its tile, so the image depends on
 * the tile grid (a splat of opacity above about 0.35 reaches 1/255 beyond
 * 3 sigma).  Without the flag the footprint is the tiles that meet the
 * ellipse o G >= 1/255, and images do not depend on the grid.  gs_render and
 * its adjoint use the footprint of the frame's last gs_project. */
#define GS_RASTER_FOOTPRINT_3SIGMA 2
/* gs_raster_opts.flags: how gs_render (gs_bin) puts each tile's list in
 * (depth bits, entry) order.  Without the flag every list is sorted on its own
 * after a radix sort of the instances by tile.  With it the visible entries
 * are radix sorted by depth first and emitted in that order, so the stable
 * sort by tile leaves every list in order with no per-tile sort.  The lists,
 * images and gradients are identical; the cost differs with the list lengths
 * (long lists favour the presort), which is what the autotuner measures. */
#define GS_RASTER_DEPTH_PRESORT 4
/* gs_raster_opts.flags: the radix sort of the instances by tile splits the
 * tile id's bits into digits of equal width (13 bits: 7 + 6) instead of 8-bit
 * digits and a narrower last one (8 + 5).  Same passes, same result; a tuning
 * knob. */
#define GS_RASTER_BALANCED_DIGITS 8
/* gs_raster_opts.flags: gs_project_backward writes the gradient rows of the
 * Gaussians some view rendered and leaves every other row as it was (their
 * gradient is zero), for callers whose optimiser reads rendered rows only
 * (gs_adam_step with the frame's tiles_touched).  Without the flag every row is
 * written. */
#define GS_RASTER_GRAD_RENDERED_ONLY 16
/* gs_raster_opts.flags: lane layout of the compositing kernels (Eq. 2 and its
 * adjoint).  A frame of fewer than 2048 tiles rendered on the plain grid gives
 * each lane one pixel (four waves per 16x16 tile, each owning an 8x8
 * quarter): such frames have at most two tiles per SIMD (1024 SIMDs), and one
 * wave per tile would run each splat step at a single wave's latency.  Larger frames, and every persistent
 * launch, give each lane a 2x2 quad (one wave per tile).  LANE_PIXELS forces
 * one pixel per lane (not with persistent_blocks > 0), LANE_QUADS forces
 * quads; setting both is an error.  Images, transmittance and walk lengths are
 * bit-identical in both layouts; the adjoint's per-splat sums are added in a
 * different order. */
#define GS_RASTER_LANE_PIXELS 32
#define GS_RASTER_LANE_QUADS 64

/* ------------------------------------------------------------------------ */
/* Frame: the device state of one rendering step for a fixed set of view     */
/* shapes (projected splats, sort buffers, tile ranges, per-pixel state,     */
/* per-splat gradients).  Its memory is a caller-owned device workspace.     */
/* ------------------------------------------------------------------------ */
typedef struct gs_frame gs_frame;

/* Bytes of device workspace a frame needs (host call, no device work).
 * n: Gaussians; n_views <= GS_MAX_VIEWS; widths/heights: host arrays of the
 * view sizes; max_instances: capacity for (view, tile, Gaussian) instances,
 * in [1, 2^30); n_views * n must be below 2^30. */
gs_status gs_frame_workspace_size(int64_t n, int32_t n_views, const int32_t* widths,
                                  const int32_t* heights, int64_t max_instances, uint64_t* bytes);

/* Create a frame over `workspace` (device, at least the queried size, 256-byte
 * aligned).  Copies a small view table to the device (synchronises). */
gs_status gs_frame_create(int64_t n, int32_t n_views, const int32_t* widths,
                          const int32_t* heights, int64_t max_instances, void* workspace,
                          uint64_t workspace_bytes, gs_frame** out);
gs_status gs_frame_destroy(gs_frame* frame);

/* Buffers inside the frame, for inspection (device pointer and element count). */
enum {
    GS_BUF_DEPTH_KEY = 0,     /* u32 [V*n]   FP32 bits of the camera depth of entry v*n+i */
    GS_BUF_TILES_TOUCHED = 1, /* u32 [V*n]   tiles covered by the footprint (0 = not rendered) */
    GS_BUF_RECT = 2,          /* u32 [V*n][2] tile rect: x0 | x1 << 16, y0 | y1 << 16 */
    GS_BUF_SPLAT = 3,         /* f32 [V*n][12] mean hi (2), mean lo (2), l11 l21 l22, opacity, rgb, pad;
                                 mean = hi + lo; [l11 0; l21 l22] is the Cholesky factor of
                                 kappa Q, Q = Sigma'^-1 the conic, kappa = log2(e)/2, so that
                                 G(d) = 2^-((l11 dx + l21 dy)^2 + (l22 dy)^2) */
    GS_BUF_VISIBLE = 4,       /* u32 [V*n]   visible entries (tiles_touched > 0), in entry order */
    GS_BUF_INST_TILE = 5,     /* u32 [cap]   tile id of each instance, in (tile, depth bits, entry) order */
    GS_BUF_INST_ENTRY = 6,    /* u32 [cap]   entry id of each instance, same order */
    GS_BUF_RANGES = 7,        /* u32 [T][2]  [start, end) of each tile's instance list */
    GS_BUF_T_FINAL = 8,       /* f32 [P]     final transmittance per pixel */
    GS_BUF_N_CONTRIB = 9,     /* u32 [P]     instances walked per pixel (last composited + 1) */
    GS_BUF_SPLAT_GRAD = 10,   /* f32 [V*n][9] dL/d(mean2d x, y, conic a, b, c, opacity, r, g, b);
                                 defined for rendered entries (tiles_touched > 0) only */
    GS_BUF_COUNTERS = 11,     /* u32 [16]    [0] visible entries, [1] instances, [2] overflow flag of
                                 the last binning, [6] sticky overflow flag: set by every binning
                                 that overflowed, cleared only by the caller (write 0), so a caller
                                 that does not read [2] after each render can check many at once */
    GS_BUF_N_COMPOSITED = 12  /* u32 [P]     splats composited per pixel */
};
gs_status gs_frame_buffer(const gs_frame* frame, int32_t which, void** ptr, int64_t* count);

/* Visible entries, instances and the overflow flag of the last render
 * (synchronises the stream).  overflow != 0 means max_instances was too small:
 * the images are incomplete; grow the frame and render again. */
gs_status gs_frame_status(gs_frame* frame, void* stream, int64_t* n_visible,
                          int64_t* n_instances, int32_t* overflow);

/* ------------------------------------------------------------------------ */
/* Rendering and its adjoint                                                 */
/* ------------------------------------------------------------------------ */

/* project(means, scales, quats, opacities, SH, camera): for every view v and
 * Gaussian i, the camera depth, the EWA screen-space Gaussian (mean, conic =
 * Sigma'^-1, opacity), its SH colour for the direction from the camera
 * centre, and its footprint rectangle in tiles.  cameras: device gs_camera[V]
 * whose width/height must equal the frame's view sizes.  g->n must equal the
 * frame's n. */
gs_status gs_project(gs_frame* frame, const gs_gaussians* g, const gs_camera* cameras,
                     const gs_raster_opts* opts, void* stream);

/* render(view, resolution): sort the projected footprints into per-tile,
 * depth-ordered lists (prefix sums, an LSD radix sort on the tile id, then
 * each tile's list ordered by (depth bits, entry)) and composite every
 * pixel of every view front to back (Eq. 2).  images: device FP32, the views'
 * planar images one after the other (sum_v 3 H_v W_v floats).  Also keeps the
 * per-pixel final transmittance and walk length for the backward. */
gs_status gs_render(gs_frame* frame, const gs_raster_opts* opts, float* images, void* stream);

/* The two halves of gs_render, for callers that time or schedule them apart.
 * gs_bin: the per-tile, depth-ordered lists of the frame's last gs_project
 * (and, with persistent_blocks > 0, the heavy-first tile order).
 * gs_composite: compositing (Eq. 2) over the lists of the frame's last gs_bin;
 * persistent_blocks > 0 needs a gs_bin that ran with persistent_blocks > 0
 * (else GS_ERR_INVALID).  gs_bin followed by gs_composite is gs_render. */
gs_status gs_bin(gs_frame* frame, const gs_raster_opts* opts, void* stream);
gs_status gs_composite(gs_frame* frame, const gs_raster_opts* opts, float* images, void* stream);

/* gs_composite with the L1 term of Eq. 3 computed as each pixel is written:
 * loss[0] += l1_scale * sum |image - target| and dL_dimages = l1_scale *
 * sign(image - target) (sign(0) = 0): gs_composite followed by
 * gs_l1_loss_grad, with the same image, the same gradient bit for bit and the
 * loss summed in another order.  targets, dL_dimages: the images' layout;
 * loss: one device float the caller has set (the call adds to it).  Errors as
 * gs_composite, and GS_ERR_INVALID for a null targets, loss or dL_dimages. */
gs_status gs_composite_l1(gs_frame* frame, const gs_raster_opts* opts, float* images,
                          const float* targets, float l1_scale, float* loss, float* dL_dimages,
                          void* stream);

/* Adjoint of gs_render: from dL/dimages (same layout as images) to the
 * per-splat gradients GS_BUF_SPLAT_GRAD, which gs_project cleared; call it
 * once per gs_project/gs_render.  Walks each pixel's list back to front,
 * recovering transmittance from the saved final value.  One kernel launch
 * (plus a one-word queue reset when persistent_blocks > 0).  persistent_blocks
 * > 0 walks the heavy-first tile order, which only a gs_render with
 * persistent_blocks > 0 builds: after a plain gs_render it is GS_ERR_INVALID. */
gs_status gs_render_backward(gs_frame* frame, const gs_raster_opts* opts,
                             const float* dL_dimages, void* stream);

/* Adjoint of gs_project (the chain rule through Sigma = R S S^T R^T,
 * Sigma' = J W Sigma W^T J^T and the SH colour of the Preliminary section):
 * from the per-splat gradients to the raw parameters, summed over the frame's
 * views (grads are overwritten, every Gaussian gets a value).  When accum and
 * denom are not NULL, also accumulates the densification statistic of the
 * Preliminary section's last paragraph (the view-space position gradient whose
 * norm selects Gaussians for densification), read as the mean over views of
 * the per-view norm: for each view where entry (v, i) was rendered,
 * accum[i] += ||(dL/dmean2d_x W_v/2, dL/dmean2d_y H_v/2)|| and denom[i] += 1. */
gs_status gs_project_backward(gs_frame* frame, const gs_gaussians* g, const gs_camera* cameras,
                              const gs_raster_opts* opts, const gs_gaussian_grads* grads,
                              float* accum, float* denom, void* stream);

/* L1 term of Eq. 3: loss[0] += scale * sum |image - target| and
 * dL_dimage = scale * sign(image - target) (sign(0) = 0). */
gs_status gs_l1_loss_grad(const float* image, const float* target, int64_t numel, float scale,
                          float* loss, float* dL_dimage, void* stream);

/* ------------------------------------------------------------------------ */
/* Densification                                                             */
/* ------------------------------------------------------------------------ */

/* accumulate_densify_stats (Preliminary, last paragraph: the view-space
 * position-gradient statistic that drives densification, as the mean over
 * views of its per-view norm in NDC units): for v in 0..n_views-1 in order, for every i with
 * visible[v][i] != 0: gx = dmean2d[v][0][i] * W_v/2, gy = dmean2d[v][1][i] * H_v/2
 * (FP32), accum[i] += sqrt(fma(gx, gx, gy*gy)) (correctly rounded), denom[i] += 1.
 * dmean2d: device [V][2][n] pixel-space gradients; visible: device int32 [V][n];
 * view_wh: HOST int32 [V][2].  Deterministic. */
gs_status gs_accumulate_densify_stats(const float* dmean2d, const int32_t* visible,
                                      const int32_t* view_wh, int32_t n_views, int64_t n,
                                      float* accum, float* denom, void* stream);

/* Which densification a selected ("hot") Gaussian receives.  ADAPTIVE is the
 * 3DGS rule of the Preliminary section's last paragraph (large ones split,
 * small ones clone); SPLIT_LARGE is the global phase of the global-to-local
 * framework (large ones split, clones suppressed); SPLIT_ONLY and CLONE_ONLY
 * are the single-operation variants the paper compares its strategy against
 * (Global-to-local framework, Gaussian distribution comparison): every hot
 * Gaussian splits, or every hot Gaussian clones.  0 and 1 keep the meaning of
 * a clone-allowed flag. */
enum {
    GS_DENSIFY_SPLIT_LARGE = 0,
    GS_DENSIFY_ADAPTIVE = 1,
    GS_DENSIFY_SPLIT_ONLY = 2,
    GS_DENSIFY_CLONE_ONLY = 3
};

/* Split / clone / prune masks (u8, 0 or 1):
 *   avg = accum/denom (0 where denom == 0), FP32 correctly rounded;
 *   hot = avg >= grad_threshold;  large = max_k log_scales[k][i] > log_scale_threshold;
 *   split = hot and (large for SPLIT_LARGE and ADAPTIVE, always for SPLIT_ONLY,
 *           never for CLONE_ONLY);
 *   clone = hot and not split, except under SPLIT_LARGE (no clones);
 *   prune = opacity_logits[i] < logit_threshold.
 * Thresholds are in raw-parameter space: log_scale_threshold = ln(rho * extent),
 * logit_threshold = ln(tau_o / (1 - tau_o)).  mode: GS_DENSIFY_*; any other
 * value is GS_ERR_INVALID. */
gs_status gs_densify_select(const float* accum, const float* denom, const float* log_scales,
                            const float* opacity_logits, int64_t n, float grad_threshold,
                            float log_scale_threshold, float logit_threshold, int32_t mode,
                            uint8_t* split, uint8_t* clone, uint8_t* prune, void* stream);

enum { GS_KIND_KEEP = 0, GS_KIND_CLONE = 1, GS_KIND_SPLIT0 = 2, GS_KIND_SPLIT1 = 3 };

/* Device workspace bytes for gs_densify_plan over n parents. */
gs_status gs_densify_plan_workspace_size(int64_t n, uint64_t* bytes);

/* densify(split_mask, clone_mask, prune_mask), step 1: the compaction map of
 * the densification rule (Preliminary, last paragraph: large Gaussians are
 * split in two, small ones cloned, transparent ones removed).
 * Parent i emits nothing if prune[i]; else [SPLIT0, SPLIT1] if split[i];
 * else [KEEP, CLONE] if clone[i]; else [KEEP].  Outputs follow parent order:
 * src[j] = parent of output row j, kind[j] = GS_KIND_*.  n_out (device int64)
 * receives the number of rows; rows beyond `capacity` are not written (then
 * n_out > capacity tells the caller to grow and call again). */
gs_status gs_densify_plan(const uint8_t* split, const uint8_t* clone, const uint8_t* prune,
                          int64_t n, int32_t* src, uint8_t* kind, int64_t capacity,
                          int64_t* n_out, void* workspace, uint64_t workspace_bytes,
                          void* stream);

/* gs_densify_plan for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same map, with the scan scratch in a fixed device array inside the library
 * instead of a workspace argument.  At most 2^23 parents per call (larger n is
 * GS_ERR_INVALID before anything is enqueued); the array takes 32 MiB of each
 * GPU the library runs on until the process ends.  The first call on a device
 * looks the array up (with that device current); no call allocates.  Every
 * call on one GPU uses the same array, so calls that overlap on one GPU (two
 * streams at once) race; calls in stream order do not. */
gs_status gs_densify_plan_noalloc(const uint8_t* split, const uint8_t* clone,
                                  const uint8_t* prune, int64_t n, int32_t* src, uint8_t* kind,
                                  int64_t capacity, int64_t* n_out, void* stream);

/* How an attribute row is produced from its parent row. */
enum {
    GS_ATTR_COPY = 0,      /* every output row copies its parent's row */
    GS_ATTR_MEAN = 1,      /* SPLITk rows: mu + R(q) (s * z_k), z_k ~ N(0, I3) from Philox; else copy */
    GS_ATTR_LOGSCALE = 2,  /* SPLITk rows: parent - ln(1.6); else copy */
    GS_ATTR_ZERO_NEW = 3,  /* KEEP rows copy, CLONE/SPLIT rows are zero (optimizer moments) */
    GS_ATTR_ZERO = 4,      /* every output row is zero (densification statistics) */
    /* Lineage counters of the Spatial diffusion analysis (Methodology): each
     * Gaussian carries its parent point's original position (GS_ATTR_COPY) and
     * the number of splits and clones on its line of descent. */
    GS_ATTR_SPLIT_COUNT = 5,  /* SPLITk rows: parent + 1; else copy */
    GS_ATTR_CLONE_COUNT = 6   /* both rows of a cloned parent (KEEP, CLONE): parent + 1; else copy */
};

/* One attribute: in [rows][n_in] -> out [rows][n_out] (device FP32). */
typedef struct {
    const float* in;
    float* out;
    int32_t rows;
    int32_t policy;
} gs_attr;

/* densify step 2: produce every attribute's new rows.  n_out: host value (the
 * caller read it to allocate).  parent_means/parent_log_scales/parent_quats are
 * the inputs [3|3|4][n_in] that GS_ATTR_MEAN needs.  The split normals for
 * child k of parent i come from Philox4x32-10 with counter
 * (i lo, i hi, k, step) and key (seed lo, seed hi): u1 = ((x0 >> 8) + 1) 2^-24,
 * u2 = (x1 >> 8) 2^-24, z0/z1 = Box-Muller cos/sin, z2 = Box-Muller cos of
 * (x2, x3).  attrs: HOST array of n_attrs <= 24. */
gs_status gs_densify_apply(const int32_t* src, const uint8_t* kind, int64_t n_out, int64_t n_in,
                           const gs_attr* attrs, int32_t n_attrs, const float* parent_means,
                           const float* parent_log_scales, const float* parent_quats,
                           uint64_t seed, uint64_t step, void* stream);

/* Spatial order of the Gaussians, a memory layout (not a step of the paper's
 * method): the permutation that sorts them by the Morton (Z-order) code of
 * their means on a 1024^3 grid over the cube of the means' bounding box (side
 * = its longest extent; cell q = min(1023, trunc((x - min) * (1024 / side))) in
 * FP32 per axis, x in the code's bit 0; non-finite means last), ties by index.
 * Output as a densification map, src[j] = the Gaussian placed at row j and
 * kind[j] = GS_KIND_KEEP (src and kind: [n]); gs_densify_apply with this map
 * gathers parameters, optimiser moments and any other per-Gaussian attribute.
 * Images are unchanged and gradients are permuted alike, while the Gaussians a
 * view renders become neighbours in memory, so the projection, its adjoint and
 * sparse Adam touch whole cache lines and skip whole waves of Gaussians that
 * no view rendered.  workspace: gs_spatial_order_workspace_size(n) bytes. */
gs_status gs_spatial_order_workspace_size(int64_t n, uint64_t* bytes);
gs_status gs_spatial_order(const float* means, int64_t n, int32_t* src, uint8_t* kind,
                           void* workspace, uint64_t workspace_bytes, void* stream);

/* The split normals of (parent, child) pairs as the apply step draws them:
 * words [m][4] (raw Philox output) and z [m][3]. */
gs_status gs_split_normals(const int64_t* parents, const int32_t* children, int64_t m,
                           uint64_t seed, uint64_t step, uint32_t* words, float* z, void* stream);

/* Adaptive opacity threshold (Methodology, Adaptive Opacity Pruning: the
 * pruning threshold is the opacity at the p-quantile, capped by an upper
 * limit), in logit space: thr[0] = min(logits_sorted[k],
 * upper_logit) where logits_sorted is the ascending order of opacity_logits
 * and k = floor(n p) is given by the caller (radix select, exact).  Then
 * prune = logit < thr.  workspace: gs_radix_select_workspace_size(n). */
gs_status gs_radix_select_workspace_size(int64_t n, uint64_t* bytes);
gs_status gs_adaptive_prune_threshold(const float* opacity_logits, int64_t n, int64_t k,
                                      float upper_logit, float* thr, void* workspace,
                                      uint64_t workspace_bytes, void* stream);

/* Eq. 3 with its D-SSIM term: loss[0] += (1 - lambda) mean|I - T| +
 * lambda (1 - mean SSIM(I, T)) and dL_dimage = its gradient w.r.t. I
 * (overwritten).  SSIM per channel with an 11 x 11 Gaussian window of standard
 * deviation 1.5, zero padding, C1 = 0.01^2, C2 = 0.03^2; means over all
 * channels and pixels.  image, target, dL_dimage: device FP32 [channels][height][width]
 * (one view); workspace: gs_ssim_workspace_size bytes of device scratch. */
gs_status gs_ssim_workspace_size(int32_t channels, int32_t height, int32_t width, uint64_t* bytes);
gs_status gs_ssim_loss_grad(const float* image, const float* target, int32_t channels,
                            int32_t height, int32_t width, float lambda, float* loss,
                            float* dL_dimage, void* workspace, uint64_t workspace_bytes,
                            void* stream);

/* ------------------------------------------------------------------------ */
/* Optimiser                                                                 */
/* ------------------------------------------------------------------------ */

/* One parameter array for gs_adam_step: param, grad, m, v are device FP32
 * [rows][n] (structure of arrays, Gaussian index fastest); lr its step size. */
typedef struct {
    float* param;
    const float* grad;
    float* m;
    float* v;
    int32_t rows;
    float lr;
} gs_adam_param;

/* Sparse Adam, the optimiser step of the accelerated 3DGS training the paper
 * builds on (Experiments, implementation details): Gaussians that no view
 * rendered (tiles_touched[v][i] == 0 for every v) keep their parameters and
 * moments (the kernel stores every element back, these unchanged, so no other
 * work may touch the arrays while it runs); the others take m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * params: HOST array of n_params <= 8 entries; tiles_touched: device u32
 * [n_views][n] (a frame's GS_BUF_TILES_TOUCHED) or NULL to update every
 * Gaussian; step >= 1 is the global step count used for the bias correction. */
gs_status gs_adam_step(const gs_adam_param* params, int32_t n_params, int64_t n,
                       const uint32_t* tiles_touched, int32_t n_views, float beta1, float beta2,
                       float eps, int64_t step, void* stream);

/* The step count of gs_adam_step_counted, kept in device memory (8-byte
 * aligned, zeroed by the caller before the first call; each call adds one to
 * step and stores the two bias-correction factors it used). */
typedef struct {
    int64_t step;
    float c1;   /* 1 / (1 - beta1^step), FP64 rounded once */
    float c2;   /* 1 / (1 - beta2^step) */
} gs_adam_counter;

/* gs_adam_step with the step count read from and advanced in device memory
 * instead of passed from the host: the same update as gs_adam_step with step
 * = counter->step + 1 (bit for bit), so a caller can capture the whole
 * training step in a graph and replay it step after step (callers whose step
 * count cannot come from the host: graph capture).  counter: device pointer;
 * calls that share it must be ordered (one stream).  The counter advances on
 * every successful call, also when n or n_params is 0. */
gs_status gs_adam_step_counted(const gs_adam_param* params, int32_t n_params, int64_t n,
                               const uint32_t* tiles_touched, int32_t n_views, float beta1,
                               float beta2, float eps, gs_adam_counter* counter, void* stream);

/* The sparse Adam step fused into gs_project_backward_adam, for each of the
 * five parameter arrays k = 0..4 (means, log_scales, quats, opacity_logits,
 * sh): param[k], the gs_gaussians' array, updated in place; m[k], v[k] its
 * moments (device FP32, same layout); lr[k] its step size.  param[k] = NULL
 * leaves array k out: its gradient goes to grads as in gs_project_backward.
 * The step count t comes from counter (device; t = counter->step + 1, the
 * count the next gs_adam_step_counted call with it takes; this call does not
 * advance it) or, when counter is NULL, from step (>= 1). */
typedef struct {
    float* param[5];
    float* m[5];
    float* v[5];
    float lr[5];
    float beta1, beta2, eps;
    const gs_adam_counter* counter;
    int64_t step;
} gs_fused_adam;

/* gs_project_backward with the sparse Adam step of gs_adam_step fused in
 * for the arrays adam selects: each Gaussian's gradient, summed over the
 * views in registers, goes straight into the update (same arithmetic, bit
 * for bit, with the frame's tiles_touched deciding which Gaussians move)
 * instead of to grads, whose pointers for those arrays are neither written
 * nor read (may be NULL); every other output is gs_project_backward's.  A
 * training step that fuses all five arrays then only advances its counter
 * (gs_adam_step_counted with no arrays).  The parameters, moments and the
 * frame's state are read and written on the stream in order; no other work
 * may touch them meanwhile.  GS_ERR_INVALID before any launch for the errors
 * of gs_project_backward, a null adam, a param[k] other than the Gaussians'
 * array k, a null moment of a selected array, a null gradient of an array not
 * selected, beta outside [0, 1), eps <= 0, step < 1 without a counter or a
 * counter not 8-byte aligned.  For the optimiser step of the accelerated 3DGS
 * training the paper builds on (Experiments, implementation details). */
gs_status gs_project_backward_adam(gs_frame* frame, const gs_gaussians* g, const gs_camera* cameras,
                                   const gs_raster_opts* opts, const gs_gaussian_grads* grads,
                                   float* accum, float* denom, const gs_fused_adam* adam,
                                   void* stream);

/* ------------------------------------------------------------------------ */
/* Primitives exposed for testing                                            */
/* ------------------------------------------------------------------------ */

/* Stable LSD radix sort of (key, value) u32 pairs on the low key_bits bits
 * (1..32).  Result in keys/vals.  n <= 2^31-1.  workspace: gs_sort_workspace_size(n). */
gs_status gs_sort_workspace_size(int64_t n, uint64_t* bytes);
gs_status gs_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int32_t key_bits,
                        void* workspace, uint64_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Captured training step (hipGraph)                                         */
/* ------------------------------------------------------------------------ */
typedef struct gs_graph gs_graph;

/* Capture project -> bin -> composite with the L1 loss/gradient
 * (gs_composite_l1) -> render backward -> project backward (+ statistics)
 * for the frame's views into a hipGraph.  The graph
 * keeps every pointer given here; the caller must keep those buffers alive and
 * unchanged in size until gs_graph_destroy.  Camera contents (device) may be
 * rewritten between launches.  loss: device float, zeroed by the graph.
 * targets/images/dL_dimages: the frame's image layout.  l1_scale multiplies
 * the L1 sum. */
gs_status gs_step_graph_create(gs_frame* frame, const gs_gaussians* g, const gs_camera* cameras,
                               const gs_raster_opts* opts, float* images, const float* targets,
                               float l1_scale, float* loss, float* dL_dimages,
                               const gs_gaussian_grads* grads, float* accum, float* denom,
                               void* stream, gs_graph** out);
gs_status gs_graph_launch(gs_graph* graph, void* stream);
gs_status gs_graph_destroy(gs_graph* graph);

#ifdef __cplusplus
}
#endif
#endif /* GSMI_H */
