"""ctypes binding of libgsmi (the C ABI in include/gsmi.h).

Argument marshalling only: every step of the rendering / densification path
runs in the HIP kernels of libgsmi.so.  PyTorch provides device memory and the
current stream.  There is no CPU fallback: when the library is missing the
calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsmi.so")
_lock = threading.Lock()
_lib = None

GS_OK, GS_ERR_INVALID, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_UNSUPPORTED = range(5)
MAX_VIEWS = 32
TILE = 16

BUF_DEPTH_KEY, BUF_TILES_TOUCHED, BUF_RECT, BUF_SPLAT, BUF_VISIBLE, BUF_INST_TILE, \
    BUF_INST_ENTRY, BUF_RANGES, BUF_T_FINAL, BUF_N_CONTRIB, BUF_SPLAT_GRAD, BUF_COUNTERS, \
    BUF_N_COMPOSITED = range(13)
KIND_KEEP, KIND_CLONE, KIND_SPLIT0, KIND_SPLIT1 = range(4)
ATTR_COPY, ATTR_MEAN, ATTR_LOGSCALE, ATTR_ZERO_NEW, ATTR_ZERO, ATTR_SPLIT_COUNT, ATTR_CLONE_COUNT = \
    range(7)
DENSIFY_SPLIT_LARGE, DENSIFY_ADAPTIVE, DENSIFY_SPLIT_ONLY, DENSIFY_CLONE_ONLY = range(4)
RASTER_COUNT_COMPOSITED = 1
RASTER_FOOTPRINT_3SIGMA = 2
RASTER_DEPTH_PRESORT = 4
RASTER_BALANCED_DIGITS = 8
RASTER_GRAD_RENDERED_ONLY = 16
RASTER_LANE_PIXELS = 32
RASTER_LANE_QUADS = 64


class GsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("gsmi status %d: %s" % (status, msg))
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class Gaussians(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("sh", ctypes.c_void_p), ("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class GaussianGrads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


class RasterOpts(ctypes.Structure):
    _fields_ = [("bg", ctypes.c_float * 3), ("near_plane", ctypes.c_float),
                ("raster_batch", ctypes.c_int32), ("persistent_blocks", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Attr(ctypes.Structure):
    _fields_ = [("inp", ctypes.c_void_p), ("out", ctypes.c_void_p), ("rows", ctypes.c_int32),
                ("policy", ctypes.c_int32)]


class AdamParam(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("rows", ctypes.c_int32), ("lr", ctypes.c_float)]


class FusedAdam(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p * 5), ("m", ctypes.c_void_p * 5),
                ("v", ctypes.c_void_p * 5), ("lr", ctypes.c_float * 5), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("counter", ctypes.c_void_p),
                ("step", ctypes.c_int64)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_U64 = ctypes.c_uint64
_F = ctypes.c_float
_PP = ctypes.POINTER(ctypes.c_void_p)

# name -> argument types (every function returns gs_status unless listed in _RET)
_SIGS = {
    "gs_last_error": [],
    "gs_version": [],
    "gs_frame_workspace_size": [_I64, _I32, _P, _P, _I64, ctypes.POINTER(_U64)],
    "gs_frame_create": [_I64, _I32, _P, _P, _I64, _P, _U64, _PP],
    "gs_frame_destroy": [_P],
    "gs_frame_buffer": [_P, _I32, _PP, ctypes.POINTER(_I64)],
    "gs_frame_status": [_P, _P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I32)],
    "gs_project": [_P, ctypes.POINTER(Gaussians), _P, ctypes.POINTER(RasterOpts), _P],
    "gs_render": [_P, ctypes.POINTER(RasterOpts), _P, _P],
    "gs_bin": [_P, ctypes.POINTER(RasterOpts), _P],
    "gs_composite": [_P, ctypes.POINTER(RasterOpts), _P, _P],
    "gs_composite_l1": [_P, ctypes.POINTER(RasterOpts), _P, _P, _F, _P, _P, _P],
    "gs_render_backward": [_P, ctypes.POINTER(RasterOpts), _P, _P],
    "gs_project_backward": [_P, ctypes.POINTER(Gaussians), _P, ctypes.POINTER(RasterOpts),
                            ctypes.POINTER(GaussianGrads), _P, _P, _P],
    "gs_project_backward_adam": [_P, ctypes.POINTER(Gaussians), _P, ctypes.POINTER(RasterOpts),
                                 ctypes.POINTER(GaussianGrads), _P, _P,
                                 ctypes.POINTER(FusedAdam), _P],
    "gs_l1_loss_grad": [_P, _P, _I64, _F, _P, _P, _P],
    "gs_accumulate_densify_stats": [_P, _P, _P, _I32, _I64, _P, _P, _P],
    "gs_densify_select": [_P, _P, _P, _P, _I64, _F, _F, _F, _I32, _P, _P, _P, _P],
    "gs_densify_plan_workspace_size": [_I64, ctypes.POINTER(_U64)],
    "gs_densify_plan": [_P, _P, _P, _I64, _P, _P, _I64, _P, _P, _U64, _P],
    "gs_densify_plan_noalloc": [_P, _P, _P, _I64, _P, _P, _I64, _P, _P],
    "gs_densify_apply": [_P, _P, _I64, _I64, ctypes.POINTER(Attr), _I32, _P, _P, _P, _U64, _U64,
                         _P],
    "gs_split_normals": [_P, _P, _I64, _U64, _U64, _P, _P, _P],
    "gs_spatial_order_workspace_size": [_I64, ctypes.POINTER(_U64)],
    "gs_spatial_order": [_P, _I64, _P, _P, _P, _U64, _P],
    "gs_ssim_workspace_size": [_I32, _I32, _I32, ctypes.POINTER(_U64)],
    "gs_ssim_loss_grad": [_P, _P, _I32, _I32, _I32, ctypes.c_float, _P, _P, _P, _U64, _P],
    "gs_adam_step": [ctypes.POINTER(AdamParam), _I32, _I64, _P, _I32, ctypes.c_float,
                     ctypes.c_float, ctypes.c_float, _I64, _P],
    "gs_adam_step_counted": [ctypes.POINTER(AdamParam), _I32, _I64, _P, _I32, ctypes.c_float,
                             ctypes.c_float, ctypes.c_float, _P, _P],
    "gs_radix_select_workspace_size": [_I64, ctypes.POINTER(_U64)],
    "gs_adaptive_prune_threshold": [_P, _I64, _I64, _F, _P, _P, _U64, _P],
    "gs_sort_workspace_size": [_I64, ctypes.POINTER(_U64)],
    "gs_sort_pairs": [_P, _P, _I64, _I32, _P, _U64, _P],
    "gs_step_graph_create": [_P, ctypes.POINTER(Gaussians), _P, ctypes.POINTER(RasterOpts), _P, _P,
                             _F, _P, _P, ctypes.POINTER(GaussianGrads), _P, _P, _P, _PP],
    "gs_graph_launch": [_P, _P],
    "gs_graph_destroy": [_P],
}
_RET = {"gs_last_error": ctypes.c_char_p, "gs_version": ctypes.c_char_p}


def exported_names():
    return list(_SIGS.keys())


def lib():
    """Load libgsmi.so (built in-tree).  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libgsmi.so is not built (%s); run __graft_entry__.build()"
                                   % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            for name, args in _SIGS.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = _RET.get(name, ctypes.c_int)
            _lib = L
    return _lib


def _check(status):
    if status != GS_OK:
        raise GsError(status, lib().gs_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def version():
    return lib().gs_version().decode()


# ----------------------------------------------------------------------------
# Parameters, cameras, options
# ----------------------------------------------------------------------------
PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def gaussians_struct(params: dict, sh_degree: int) -> Gaussians:
    for k in PARAM_NAMES:
        t = params[k]
        if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("%s must be a contiguous float32 CUDA tensor" % k)
    n = params["means"].shape[-1]
    return Gaussians(params["means"].data_ptr(), params["log_scales"].data_ptr(),
                     params["quats"].data_ptr(), params["opacity_logits"].data_ptr(),
                     params["sh"].data_ptr(), n, sh_degree, 0)


def grads_struct(grads: dict) -> GaussianGrads:
    return GaussianGrads(*(grads[k].data_ptr() for k in PARAM_NAMES))


def camera_array(cams) -> np.ndarray:
    """Pack synth.Camera objects into gs_camera structs (host bytes)."""
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].R[:] = [float(x) for x in np.asarray(c.R, np.float64).reshape(9)]
        arr[i].t[:] = [float(x) for x in np.asarray(c.t, np.float64).reshape(3)]
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = c.fx, c.fy, c.cx, c.cy
        arr[i].width, arr[i].height = c.width, c.height
    return np.frombuffer(bytes(arr), np.uint8)


def cameras_to_device(cams, device="cuda") -> torch.Tensor:
    return torch.from_numpy(camera_array(cams).copy()).to(device)


def raster_opts(bg=(0.0, 0.0, 0.0), near_plane=0.2, raster_batch=0, persistent_blocks=0,
                count_composited=False, footprint_3sigma=False, depth_presort=False,
                balanced_digits=False, grad_rendered_only=False, lanes=None):
    """footprint_3sigma: bin by 3-sigma squares as the original 3DGS
    rasterizer does (images then depend on the tile grid) instead of by the
    opacity-aware ellipse (GS_RASTER_FOOTPRINT_3SIGMA).  depth_presort: order
    the visible entries by depth before emission instead of sorting each tile's
    list (GS_RASTER_DEPTH_PRESORT; same lists, different cost).  lanes: None
    (one pixel per lane for frames of fewer than 2048 tiles on the plain grid,
    a 2x2 quad otherwise), "pixels" or "quads" to force one layout."""
    if lanes not in (None, "pixels", "quads"):
        raise ValueError("lanes must be None, 'pixels' or 'quads'")
    o = RasterOpts()
    o.bg[:] = [float(x) for x in bg]
    o.near_plane = float(np.float32(near_plane))
    o.raster_batch = int(raster_batch)
    o.persistent_blocks = int(persistent_blocks)
    o.flags = ((RASTER_COUNT_COMPOSITED if count_composited else 0) |
               (RASTER_FOOTPRINT_3SIGMA if footprint_3sigma else 0) |
               (RASTER_DEPTH_PRESORT if depth_presort else 0) |
               (RASTER_BALANCED_DIGITS if balanced_digits else 0) |
               (RASTER_GRAD_RENDERED_ONLY if grad_rendered_only else 0) |
               (RASTER_LANE_PIXELS if lanes == "pixels" else 0) |
               (RASTER_LANE_QUADS if lanes == "quads" else 0))
    return o


# ----------------------------------------------------------------------------
# Frame
# ----------------------------------------------------------------------------
class Frame:
    """Device state of one rendering step for fixed view sizes (C ABI gs_frame)."""

    def __init__(self, n: int, sizes, max_instances: int, device="cuda"):
        self.n = int(n)
        self.sizes = [(int(w), int(h)) for w, h in sizes]
        self.V = len(self.sizes)
        self.cap = int(max_instances)
        self.device = torch.device(device)
        W = np.array([w for w, _ in self.sizes], np.int32)
        H = np.array([h for _, h in self.sizes], np.int32)
        self._W, self._H = W, H
        nbytes = ctypes.c_uint64()
        _check(lib().gs_frame_workspace_size(self.n, self.V, W.ctypes.data_as(_P),
                                             H.ctypes.data_as(_P), self.cap,
                                             ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(lib().gs_frame_create(self.n, self.V, W.ctypes.data_as(_P), H.ctypes.data_as(_P),
                                     self.cap, _ptr(self.workspace), int(nbytes.value),
                                     ctypes.byref(h)))
        self.handle = h
        self.tiles = [((w + TILE - 1) // TILE) * ((h + TILE - 1) // TILE) for w, h in self.sizes]
        self.pixels = [w * h for w, h in self.sizes]
        self.T = sum(self.tiles)
        self.P = sum(self.pixels)

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None and _lib is not None:
                _lib.gs_frame_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def buffer(self, which: int, dtype=torch.int32) -> torch.Tensor:
        """A view of one frame buffer (no copy)."""
        p = ctypes.c_void_p()
        cnt = ctypes.c_int64()
        _check(lib().gs_frame_buffer(self.handle, which, ctypes.byref(p), ctypes.byref(cnt)))
        elem = torch.empty(0, dtype=dtype).element_size()
        off = p.value - self.workspace.data_ptr()
        return self.workspace[off:off + cnt.value * elem].view(dtype)

    def status(self, stream=None, raise_on_overflow=True):
        nv, ni, ov = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        st = lib().gs_frame_status(self.handle, _stream(stream), ctypes.byref(nv), ctypes.byref(ni),
                                   ctypes.byref(ov))
        if st not in (GS_OK, GS_ERR_CAPACITY) or (st == GS_ERR_CAPACITY and raise_on_overflow):
            _check(st)
        return int(nv.value), int(ni.value), int(ov.value)

    def image_numel(self):
        return 3 * self.P

    def split_images(self, flat: torch.Tensor):
        """Per-view [3, H, W] views of a flat image buffer (one split, so the
        gradient of all views is gathered back with a single concatenation)."""
        parts = torch.split(flat, [3 * w * h for (w, h) in self.sizes])
        return [t.view(3, h, w) for t, (w, h) in zip(parts, self.sizes)]

    def project(self, params, sh_degree, cams_dev, opts, stream=None):
        g = gaussians_struct(params, sh_degree)
        _check(lib().gs_project(self.handle, ctypes.byref(g), _ptr(cams_dev), ctypes.byref(opts),
                                _stream(stream)))

    def render(self, opts, images=None, stream=None):
        if images is None:
            images = torch.empty(self.image_numel(), dtype=torch.float32, device=self.device)
        _check(lib().gs_render(self.handle, ctypes.byref(opts), _ptr(images), _stream(stream)))
        return images

    def bin(self, opts, stream=None):
        _check(lib().gs_bin(self.handle, ctypes.byref(opts), _stream(stream)))

    def composite(self, opts, images=None, stream=None):
        if images is None:
            images = torch.empty(self.image_numel(), dtype=torch.float32, device=self.device)
        _check(lib().gs_composite(self.handle, ctypes.byref(opts), _ptr(images), _stream(stream)))
        return images

    def composite_l1(self, opts, images, targets, scale, loss, grad, stream=None):
        """composite with the L1 term fused (gs_composite_l1): writes images,
        adds scale * sum |images - targets| to loss[0] and writes
        grad = scale * sign(images - targets)."""
        for t in (images, targets, grad):
            if t.numel() != self.image_numel() or not t.is_contiguous():
                raise ValueError("images, targets and grad must hold the frame's images")
        _check(lib().gs_composite_l1(self.handle, ctypes.byref(opts), _ptr(images), _ptr(targets),
                                     float(scale), _ptr(loss), _ptr(grad), _stream(stream)))
        return images

    def overflowed(self, clear=False):
        """Whether any binning of this frame overflowed its instance capacity
        since the flag was last cleared (reads a device word: synchronises)."""
        c = self.buffer(BUF_COUNTERS)
        flag = int(c[6].item())
        if clear:
            c[6:7].zero_()
        return flag != 0

    def render_backward(self, opts, dL_dimages, stream=None):
        _check(lib().gs_render_backward(self.handle, ctypes.byref(opts), _ptr(dL_dimages),
                                        _stream(stream)))

    def project_backward(self, params, sh_degree, cams_dev, opts, grads, accum=None, denom=None,
                         stream=None, adam=None):
        """adam: None, or the sparse Adam step to fuse in
        (gs_project_backward_adam; see FusedAdamStep): the parameter arrays it
        names are updated in place and get no gradient (grads may omit them
        or hold None)."""
        g = gaussians_struct(params, sh_degree)
        gr = GaussianGrads(*(grads[k].data_ptr() if grads.get(k) is not None else None
                             for k in PARAM_NAMES))
        if adam is None:
            _check(lib().gs_project_backward(self.handle, ctypes.byref(g), _ptr(cams_dev),
                                             ctypes.byref(opts), ctypes.byref(gr), _ptr(accum),
                                             _ptr(denom), _stream(stream)))
            return
        a = adam.struct(params)
        _check(lib().gs_project_backward_adam(self.handle, ctypes.byref(g), _ptr(cams_dev),
                                              ctypes.byref(opts), ctypes.byref(gr), _ptr(accum),
                                              _ptr(denom), ctypes.byref(a), _stream(stream)))


class FusedAdamStep:
    """The sparse Adam step a projection adjoint applies itself
    (gs_project_backward_adam).  moments: {name: (m, v)} for the parameter
    arrays to update (names of PARAM_NAMES), lrs: {name: step size}, step: a
    device counter of adam_counter (read, not advanced: a gs_adam_step_counted
    call, with the other arrays or none, advances it) or the step count from 1."""

    def __init__(self, moments, lrs, step, beta1=0.9, beta2=0.999, eps=1e-15):
        for k in moments:
            if k not in PARAM_NAMES:
                raise ValueError("unknown parameter array %r" % k)
        if isinstance(step, torch.Tensor) and (step.dtype != torch.int64 or step.numel() != 2 or
                                               not step.is_contiguous()):
            raise ValueError("step counter must be adam_counter's int64 [2] tensor")
        self.moments = dict(moments)
        self.lrs = {k: float(lrs[k]) for k in moments}
        self.step = step
        self.beta1, self.beta2, self.eps = float(beta1), float(beta2), float(eps)

    def names(self):
        return list(self.moments)

    def struct(self, params) -> FusedAdam:
        a = FusedAdam()
        for i, k in enumerate(PARAM_NAMES):
            if k not in self.moments:
                continue
            m, v = self.moments[k]
            p = params[k]
            for t in (m, v):
                if t.numel() != p.numel() or not t.is_contiguous() or t.dtype != torch.float32:
                    raise ValueError("the moments of %s must be contiguous float32 like it" % k)
            a.param[i], a.m[i], a.v[i] = p.data_ptr(), m.data_ptr(), v.data_ptr()
            a.lr[i] = self.lrs[k]
        a.beta1, a.beta2, a.eps = self.beta1, self.beta2, self.eps
        counted = isinstance(self.step, torch.Tensor)
        a.counter = self.step.data_ptr() if counted else None
        a.step = 0 if counted else int(self.step)
        return a


def empty_grads(params: dict) -> dict:
    return {k: torch.empty_like(params[k]) for k in PARAM_NAMES}


# ----------------------------------------------------------------------------
# Loss
# ----------------------------------------------------------------------------
def l1_loss_grad(image, target, scale, loss=None, grad=None, stream=None):
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=image.device)
    if grad is None:
        grad = torch.empty_like(image)
    _check(lib().gs_l1_loss_grad(_ptr(image), _ptr(target), image.numel(), float(scale),
                                 _ptr(loss), _ptr(grad), _stream(stream)))
    return loss, grad


# ----------------------------------------------------------------------------
# Densification
# ----------------------------------------------------------------------------
def accumulate_densify_stats(dmean2d, visible, view_wh, accum, denom, stream=None):
    V, _, n = dmean2d.shape
    wh = np.ascontiguousarray(np.asarray(view_wh, np.int32).reshape(V, 2))
    _check(lib().gs_accumulate_densify_stats(_ptr(dmean2d), _ptr(visible), wh.ctypes.data_as(_P),
                                             V, n, _ptr(accum), _ptr(denom), _stream(stream)))


def densify_select(accum, denom, log_scales, logits, grad_threshold, log_scale_threshold,
                   logit_threshold, mode=DENSIFY_ADAPTIVE, stream=None):
    """Split / clone / prune masks.  mode: DENSIFY_* (a bool reads as clones
    allowed: True = DENSIFY_ADAPTIVE, False = DENSIFY_SPLIT_LARGE)."""
    n = accum.numel()
    dev = accum.device
    split = torch.empty(n, dtype=torch.uint8, device=dev)
    clone = torch.empty(n, dtype=torch.uint8, device=dev)
    prune = torch.empty(n, dtype=torch.uint8, device=dev)
    _check(lib().gs_densify_select(_ptr(accum), _ptr(denom), _ptr(log_scales), _ptr(logits), n,
                                   float(grad_threshold), float(log_scale_threshold),
                                   float(logit_threshold), int(mode), _ptr(split),
                                   _ptr(clone), _ptr(prune), _stream(stream)))
    return split, clone, prune


def densify_plan(split, clone, prune, capacity=None, stream=None):
    """Returns (src, kind, n_out) -- n_out read back from the device (synchronises)."""
    n = split.numel()
    dev = split.device
    if capacity is None:
        capacity = 2 * n
    nb = ctypes.c_uint64()
    _check(lib().gs_densify_plan_workspace_size(n, ctypes.byref(nb)))
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    src = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    kind = torch.empty(max(capacity, 1), dtype=torch.uint8, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib().gs_densify_plan(_ptr(split), _ptr(clone), _ptr(prune), n, _ptr(src), _ptr(kind),
                                 capacity, _ptr(n_out), _ptr(ws), int(nb.value), _stream(stream)))
    m = plan_rows_checked(int(n_out.item()), capacity)
    return src[:m], kind[:m], m


def densify_plan_noalloc(split, clone, prune, src, kind, n_out, stream=None):
    """gs_densify_plan_noalloc into caller-provided src/kind (capacity = their
    length) and n_out (device int64[1]); nothing is allocated or synchronised."""
    n = split.numel()
    _check(lib().gs_densify_plan_noalloc(_ptr(split), _ptr(clone), _ptr(prune), n, _ptr(src),
                                         _ptr(kind), min(src.numel(), kind.numel()), _ptr(n_out),
                                         _stream(stream)))


def plan_rows_checked(n_out: int, capacity: int) -> int:
    """The plan's row count, or an error when the map did not fit: rows past
    the capacity are not written, so src/kind would be incomplete."""
    if n_out > capacity:
        raise GsError(GS_ERR_CAPACITY, "densify plan has %d rows but capacity is %d; call again "
                      "with capacity >= %d" % (n_out, capacity, n_out))
    return n_out


def densify_apply(src, kind, n_in, attrs, parent_means, parent_log_scales, parent_quats, seed,
                  step, stream=None):
    """attrs: list of (input tensor [rows, n_in] or None, rows, policy); returns outputs."""
    n_out = src.numel()
    dev = src.device
    outs = []
    arr = (Attr * len(attrs))()
    for i, (inp, rows, policy) in enumerate(attrs):
        out = torch.empty((rows, n_out), dtype=torch.float32, device=dev)
        outs.append(out)
        arr[i].inp = inp.data_ptr() if inp is not None else None
        arr[i].out = out.data_ptr()
        arr[i].rows = rows
        arr[i].policy = policy
    _check(lib().gs_densify_apply(_ptr(src), _ptr(kind), n_out, n_in, arr, len(attrs),
                                  _ptr(parent_means), _ptr(parent_log_scales), _ptr(parent_quats),
                                  int(seed), int(step), _stream(stream)))
    return outs


def spatial_order(means, stream=None):
    """(src, kind): the Morton-order permutation of the Gaussians as a map for
    densify_apply (every row KEEP)."""
    n = means.shape[-1]
    nb = ctypes.c_uint64()
    _check(lib().gs_spatial_order_workspace_size(n, ctypes.byref(nb)))
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=means.device)
    src = torch.empty(max(n, 1), dtype=torch.int32, device=means.device)
    kind = torch.empty(max(n, 1), dtype=torch.uint8, device=means.device)
    _check(lib().gs_spatial_order(_ptr(means), n, _ptr(src), _ptr(kind), _ptr(ws), int(nb.value),
                                  _stream(stream)))
    return src[:n], kind[:n]


def reorder(tensors, src, kind, stream=None):
    """Apply a spatial order (or any all-KEEP map) to [rows, n] / [n] tensors:
    one gather launch for all of them.  Returns the new tensors."""
    n = src.numel()
    attrs = [(t.reshape(-1, n), t.numel() // n, ATTR_COPY) for t in tensors]
    outs = densify_apply(src, kind, n, attrs, None, None, None, 0, 0, stream=stream)
    return [o.view(t.shape) for o, t in zip(outs, tensors)]


def split_normals(parents, children, seed, step, stream=None):
    m = parents.numel()
    words = torch.empty((m, 4), dtype=torch.int32, device=parents.device)
    z = torch.empty((m, 3), dtype=torch.float32, device=parents.device)
    _check(lib().gs_split_normals(_ptr(parents), _ptr(children), m, int(seed), int(step),
                                  _ptr(words), _ptr(z), _stream(stream)))
    return words, z


def adaptive_prune_threshold(logits, p=0.03, tau_u=0.05, stream=None):
    """tau = min(alpha_sorted[floor(N p)], tau_u) in logit space (radix select on the GPU)."""
    n = logits.numel()
    k = min(int(math.floor(n * p)), n - 1)
    upper = float(np.float32(math.log(tau_u / (1.0 - tau_u))))
    nb = ctypes.c_uint64()
    _check(lib().gs_radix_select_workspace_size(n, ctypes.byref(nb)))
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=logits.device)
    thr = torch.empty(1, dtype=torch.float32, device=logits.device)
    _check(lib().gs_adaptive_prune_threshold(_ptr(logits), n, k, upper, _ptr(thr), _ptr(ws),
                                             int(nb.value), _stream(stream)))
    return thr, k


def ssim_workspace_bytes(channels, height, width):
    nb = ctypes.c_uint64()
    _check(lib().gs_ssim_workspace_size(int(channels), int(height), int(width), ctypes.byref(nb)))
    return int(nb.value)


def ssim_loss_grad(image, target, lam=0.2, loss=None, grad=None, workspace=None, stream=None):
    """(1 - lam) L1 + lam (1 - SSIM) of one [C, H, W] image and its gradient."""
    C, H, W = image.shape
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=image.device)
    if grad is None:
        grad = torch.empty_like(image)
    nb = ctypes.c_uint64()
    _check(lib().gs_ssim_workspace_size(C, H, W, ctypes.byref(nb)))
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=image.device)
    _check(lib().gs_ssim_loss_grad(_ptr(image), _ptr(target), C, H, W, float(lam), _ptr(loss),
                                   _ptr(grad), _ptr(workspace), int(nb.value), _stream(stream)))
    return loss, grad


def adam_counter(device):
    """A zeroed gs_adam_counter on the device (int64 [2]: the step count, then
    the two FP32 bias-correction factors of the last counted step)."""
    return torch.zeros(2, dtype=torch.int64, device=device)


def adam_step(entries, n, step, tiles_touched=None, n_views=1, beta1=0.9, beta2=0.999, eps=1e-15,
              stream=None):
    """Sparse Adam step.  entries: list of (param, grad, m, v, lr), tensors of
    shape [rows, n] (or [n]); tiles_touched: a frame's BUF_TILES_TOUCHED (only
    Gaussians rendered in some view are updated) or None (all of them).
    step: the global step count (from 1), or a device counter of adam_counter,
    which the call advances on the device (gs_adam_step_counted)."""
    arr = (AdamParam * len(entries))()
    for i, (p, g, m, v, lr) in enumerate(entries):
        rows = p.numel() // n if n else 0
        for t in (g, m, v):
            if t.numel() != p.numel() or not t.is_contiguous():
                raise ValueError("grad and moments must match the parameter's shape")
        arr[i].param, arr[i].grad, arr[i].m, arr[i].v = (p.data_ptr(), g.data_ptr(), m.data_ptr(),
                                                         v.data_ptr())
        arr[i].rows = rows
        arr[i].lr = float(lr)
    if isinstance(step, torch.Tensor):
        if step.dtype != torch.int64 or step.numel() != 2 or not step.is_contiguous():
            raise ValueError("step counter must be adam_counter's int64 [2] tensor")
        _check(lib().gs_adam_step_counted(arr, len(entries), int(n), _ptr(tiles_touched),
                                          int(n_views), float(beta1), float(beta2), float(eps),
                                          _ptr(step), _stream(stream)))
        return
    _check(lib().gs_adam_step(arr, len(entries), int(n), _ptr(tiles_touched), int(n_views),
                              float(beta1), float(beta2), float(eps), int(step), _stream(stream)))


def sort_pairs(keys, vals, key_bits=32, stream=None):
    """In-place stable radix sort of int32-viewed u32 keys/values on the GPU."""
    n = keys.numel()
    nb = ctypes.c_uint64()
    _check(lib().gs_sort_workspace_size(n, ctypes.byref(nb)))
    ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=keys.device)
    _check(lib().gs_sort_pairs(_ptr(keys), _ptr(vals), n, int(key_bits), _ptr(ws), int(nb.value),
                               _stream(stream)))


# ----------------------------------------------------------------------------
# Captured step
# ----------------------------------------------------------------------------
class StepGraph:
    """hipGraph of project -> bin -> composite with the L1 term -> render
    backward -> project backward."""

    def __init__(self, frame: Frame, params, sh_degree, cams_dev, opts, images, targets, l1_scale,
                 loss, dL, grads, accum=None, denom=None, stream=None):
        self._keep = (frame, params, cams_dev, images, targets, loss, dL, grads, accum, denom)
        g = gaussians_struct(params, sh_degree)
        gr = grads_struct(grads)
        h = ctypes.c_void_p()
        _check(lib().gs_step_graph_create(frame.handle, ctypes.byref(g), _ptr(cams_dev),
                                          ctypes.byref(opts), _ptr(images), _ptr(targets),
                                          float(l1_scale), _ptr(loss), _ptr(dL), ctypes.byref(gr),
                                          _ptr(accum), _ptr(denom), _stream(stream),
                                          ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(lib().gs_graph_launch(self.handle, _stream(stream)))

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None and _lib is not None:
                _lib.gs_graph_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
