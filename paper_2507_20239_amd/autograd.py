"""torch.autograd wrapper of the rasterizer (projection + binning +
compositing forward, compositing adjoint + projection adjoint backward).

The forward keeps no per-(pixel, splat) state: what the backward needs is the
frame's projected splats, sorted tile lists, tile ranges and per-pixel final
transmittance and walk length, all inside the frame workspace; the adjoint
kernel recomputes every alpha and transmittance from them (back-to-front replay).
The densification statistic (mean over views of the view-space position
gradient norm, Preliminary, last paragraph of the paper) accumulates into the
rasterizer's `accum` / `denom` as a side effect of the backward.

Every step of the computation runs in libgsmi.so; this module only moves
pointers.  A frame holds the state of one forward at a time: calling the
rasterizer again before the backward of an earlier call invalidates that
backward, which then raises instead of returning wrong gradients.
"""
import types

import torch

from . import autotune, gsmi


class GaussianRasterizer:
    """Renders N Gaussians into a fixed list of views.

    cameras: list of objects with R (3x3), t (3), fx, fy, cx, cy, width, height
    (see synth.Camera); their sizes fix the frame.  The instance capacity
    grows (and the step re-runs) when a render overflows it.  footprint_3sigma
    bins by the original 3DGS 3-sigma squares (gsmi.raster_opts).
    raster_batch, persistent_blocks, depth_presort, balanced_digits and lanes
    set the launch shape (gsmi.raster_opts).  With autotune=True the first
    call times the autotuner's launch shapes (LDS batch, lane layout or
    heavy-first persistent grid, sort form, digit split) on these views and
    parameters and keeps the fastest instead.
    """

    def __init__(self, n, cameras, sh_degree, device="cuda", bg=(0.0, 0.0, 0.0),
                 raster_batch=0, persistent_blocks=0, capacity=None, near_plane=0.2,
                 footprint_3sigma=False, autotune=False, lazy_overflow=False,
                 depth_presort=False, balanced_digits=False, lanes=None):
        self.n = int(n)
        self.sh_degree = int(sh_degree)
        self.device = torch.device(device)
        # lazy_overflow: the forward does not read the overflow flag back (no host
        # synchronisation per call); the caller checks overflowed() when it
        # chooses and repeats the affected steps with a larger capacity (grow())
        self.lazy_overflow = bool(lazy_overflow)
        self._opt_args = dict(bg=bg, near_plane=near_plane, footprint_3sigma=footprint_3sigma)
        self.opts = gsmi.raster_opts(raster_batch=raster_batch, persistent_blocks=persistent_blocks,
                                     depth_presort=depth_presort, balanced_digits=balanced_digits,
                                     lanes=lanes, **self._opt_args)
        self.autotune = bool(autotune)
        self.tuned = None
        self.set_cameras(cameras)
        sizes = [(c.width, c.height) for c in cameras]
        if capacity is None:
            tiles = sum(((w + 15) // 16) * ((h + 15) // 16) for w, h in sizes)
            capacity = max(1 << 20, 64 * tiles)
        self.frame = gsmi.Frame(self.n, sizes, capacity, self.device)
        self.accum = torch.zeros(self.n, device=self.device)
        self.denom = torch.zeros(self.n, device=self.device)
        self.generation = 0
        self.adam = None

    def fuse_adam(self, adam):
        """Fuse a sparse Adam step into the backward (a gsmi.FusedAdamStep, or
        None to switch fusion off; gs_project_backward_adam): the backward
        updates the parameter tensors it names in place, with their moments,
        and returns no gradient for them.  The caller's optimiser step covers
        the others, and with a device step counter advances it (a counted
        gsmi.adam_step with the remaining arrays, or none).  Same bits as a
        separate gsmi.adam_step."""
        self.adam = adam

    def set_cameras(self, cameras):
        """New poses / intrinsics for views of the same sizes."""
        if hasattr(self, "frame"):
            sizes = [(c.width, c.height) for c in cameras]
            if sizes != self.frame.sizes:
                raise ValueError("view sizes differ from the frame's; build a new rasterizer")
        self.cameras = list(cameras)
        self.cams_dev = gsmi.cameras_to_device(self.cameras, self.device)

    def use_device_cameras(self, cams_dev):
        """Cameras already packed on the device (gs_camera rows, e.g. rows of
        gsmi.cameras_to_device of a larger table indexed on the device), so a
        training loop can change views without a host-to-device copy.  The
        views must have the frame's sizes; that is the caller's contract."""
        if cams_dev.numel() != self.cams_dev.numel() or cams_dev.device != self.cams_dev.device:
            raise ValueError("expected %d bytes of cameras on %s"
                             % (self.cams_dev.numel(), self.cams_dev.device))
        self.cams_dev = cams_dev.contiguous()

    def overflowed(self, clear=True):
        """Whether any forward since the last check overflowed the instance
        capacity (synchronises).  Only needed with lazy_overflow=True."""
        return self.frame.overflowed(clear=clear)

    def grow(self, factor=2):
        self._grow(self.frame.cap * factor)

    def reset_stats(self):
        self.accum.zero_()
        self.denom.zero_()

    def _tune(self, params):
        """Pick the launch shape by timing the autotuner's candidates."""
        scene = types.SimpleNamespace(n=self.n, sh_degree=self.sh_degree)
        best = autotune.tune_batched(scene, self.cameras, params, self.device, cap=self.frame.cap,
                                     opts=self._opt_args)
        self.opts = autotune.opts_of(best, **self._opt_args)
        self.tuned = best

    def _grow(self, needed):
        cap = self.frame.cap
        while cap < needed:
            cap *= 2
        self.frame = gsmi.Frame(self.n, self.frame.sizes, cap, self.device)

    def __call__(self, means, log_scales, quats, opacity_logits, sh):
        """Images of every view, as a list of [3, H, W] tensors (differentiable
        w.r.t. all five parameter tensors)."""
        flat = _Rasterize.apply(means, log_scales, quats, opacity_logits, sh, self)
        return self.frame.split_images(flat)


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, r):
        params = {"means": means.detach().contiguous(), "log_scales": log_scales.detach().contiguous(),
                  "quats": quats.detach().contiguous(),
                  "opacity_logits": opacity_logits.detach().contiguous(),
                  "sh": sh.detach().contiguous()}
        for k, t in params.items():
            if t.dtype != torch.float32 or t.device != r.device:
                raise TypeError("%s must be float32 on %s" % (k, r.device))
        tune = r.autotune and r.tuned is None
        while True:
            r.frame.project(params, r.sh_degree, r.cams_dev, r.opts)
            images = r.frame.render(r.opts)
            if r.lazy_overflow and not tune:
                break
            nv, ni, ovf = r.frame.status(raise_on_overflow=False)
            if not ovf:
                if not tune:
                    break
                # the capacity now holds the step: time the candidates, then
                # render once more with the chosen shape
                r._tune(params)
                tune = False
                continue
            r._grow(ni)
        r.generation += 1
        ctx.r = r
        ctx.generation = r.generation
        ctx.params = params
        ctx.cams_dev = r.cams_dev
        ctx.adam = r.adam
        if r.adam is not None:
            given = dict(means=means, log_scales=log_scales, quats=quats,
                         opacity_logits=opacity_logits, sh=sh)
            for k in r.adam.names():
                if params[k].data_ptr() != given[k].data_ptr():
                    raise ValueError("a fused Adam step updates %s in place: it must be "
                                     "contiguous" % k)
        return images

    @staticmethod
    def backward(ctx, dL_dimages):
        r = ctx.r
        if r.generation != ctx.generation:
            raise RuntimeError("the rasterizer rendered again before this backward; its frame no "
                               "longer holds this forward's state")
        r.frame.render_backward(r.opts, dL_dimages.contiguous())
        fused = ctx.adam.names() if ctx.adam is not None else []
        grads = {k: None if k in fused else torch.empty_like(ctx.params[k])
                 for k in gsmi.PARAM_NAMES}
        r.frame.project_backward(ctx.params, r.sh_degree, ctx.cams_dev, r.opts, grads, r.accum,
                                 r.denom, adam=ctx.adam)
        return (grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logits"],
                grads["sh"], None)


class _PhotometricLoss(torch.autograd.Function):
    """Eq. 3 of one view, (1 - lambda) L1 + lambda D-SSIM, with its gradient
    computed in the same kernel launches as the loss (gs_ssim_loss_grad)."""

    @staticmethod
    def forward(ctx, image, target, lam, workspace):
        loss = torch.zeros(1, dtype=torch.float32, device=image.device)
        loss, grad = gsmi.ssim_loss_grad(image.contiguous(), target.contiguous(), lam, loss=loss,
                                         workspace=workspace)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g, None, None, None


def photometric_loss(image, target, lam=0.2, workspace=None):
    """Differentiable Eq. 3 loss of a [3, H, W] image against its target.
    workspace: optional uint8 device buffer of gsmi.ssim_workspace_bytes."""
    return _PhotometricLoss.apply(image, target, float(lam), workspace)
