"""FP64 CPU oracle: a plain, slow, obviously correct reference for the
Gaussian-splatting hot path (projection, per-pixel compositing, its adjoint,
the densification statistic, the split/clone/prune compaction, Philox split
sampling, adaptive opacity threshold).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this package.  It shares no code with the GPU
library: the C part (oracle.c) is compiled here with gcc, and nothing in the
GPU package imports it.  Inputs are the same FP32 arrays the GPU receives,
widened exactly to double.

Paper: "Decomposing Densification in Gaussian Splatting for Faster 3D Scene
Reconstruction".  Passages: Eq. 1 and the Sigma / Sigma' definitions
(Preliminary), Eq. 2 (compositing), the densification rule (Preliminary, last
paragraph), global-to-local phases (Methodology, Global-to-local framework),
Eqs. 4-6 (coarse-to-fine schedule), adaptive opacity threshold (Methodology,
Adaptive Opacity Pruning).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "_oracle.so")
_lock = threading.Lock()
_lib = None

NEAR_PLANE = float(np.float32(0.2))
TILE = 16


def build(force: bool = True) -> str:
    """Compile oracle.c into oracle/_oracle.so with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            _lib = ctypes.CDLL(_LIB_PATH)
            _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double
_F = ctypes.c_float
_U64 = ctypes.c_uint64


def _declare(L):
    L.oracle_sh_basis.argtypes = [ctypes.c_int, _P, _P, _P]
    L.oracle_project.argtypes = [_I64, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_int,
                                 ctypes.c_int, _D] + [_P] * 10
    L.oracle_render_pixels.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _P, _P]
    L.oracle_render_backward_pixels.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _I64, _P, _P, _P,
                                                _P, _P]
    L.oracle_project_backward.argtypes = [_I64, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_int,
                                          ctypes.c_int, _D, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.oracle_philox4x32_10.argtypes = [_P, _P, _P]
    L.oracle_split_normals.argtypes = [_U64, _U64, _I64, ctypes.c_int, _P, _P]
    L.oracle_split_means.argtypes = [_I64, _P, _P, _P, _I64, _P, _P, _U64, _U64, _P]
    L.oracle_stats_f32.argtypes = [_I64, _I32, _P, _P, _P, _P, _P]
    L.oracle_select.argtypes = [_I64, _P, _P, _P, _P, _F, _F, _F, ctypes.c_int, _P, _P, _P]
    L.oracle_covariance3d.argtypes = [_P, _P, _P]
    L.oracle_set_threads.argtypes = [ctypes.c_int]
    L.oracle_max_threads.restype = ctypes.c_int


def set_threads(threads: int) -> None:
    """Thread count of the oracle's OpenMP loops (results do not depend on it)."""
    lib().oracle_set_threads(int(threads))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype))


# ----------------------------------------------------------------------------
# Spherical harmonics and covariance
# ----------------------------------------------------------------------------
def sh_basis(deg: int, direction):
    """Real SH (Condon-Shortley phase) Y[k], k = l^2 + l + m, and the gradient
    of their polynomial form w.r.t. (x, y, z) at a unit direction."""
    d = _c(direction, np.float64)
    K = (deg + 1) ** 2
    Y = np.zeros(16)
    dY = np.zeros(48)
    lib().oracle_sh_basis(deg, _ptr(d), _ptr(Y), _ptr(dY))
    return Y[:K].copy(), dY[:3 * K].reshape(K, 3).copy()


def covariance3d(quat, log_scale):
    q = _c(quat, np.float64)
    s = _c(log_scale, np.float64)
    S = np.zeros(9)
    lib().oracle_covariance3d(_ptr(q), _ptr(s), _ptr(S))
    return S.reshape(3, 3)


# ----------------------------------------------------------------------------
# Projection (Preliminary: Sigma and Sigma' = J W Sigma W^T J^T; Eq. 2's colour)
# ----------------------------------------------------------------------------
def camera_array(cam) -> np.ndarray:
    return _c(cam.as_floats(), np.float64)


def project(scene_or_params, cam, near_plane: float = NEAR_PLANE, footprint: str = "ellipse") -> dict:
    """Project every Gaussian into one camera (FP64).  tiles_touched counts the
    tiles footprint_tiles bins a Gaussian to; flags bit 0 also marks Gaussians
    with a tile decision within rounding distance of flipping.  footprint:
    "ellipse" (the tiles meeting o G >= 1/255) or "3sigma" (the tiles meeting
    the 3-sigma square, whatever the opacity; see footprint_3sigma)."""
    p = scene_or_params
    n = int(p.means.shape[1])
    deg = int(p.sh_degree)
    means = _c(p.means, np.float32)
    ls = _c(p.log_scales, np.float32)
    q = _c(p.quats, np.float32)
    lg = _c(p.opacity_logits, np.float32)
    sh = _c(p.sh, np.float32)
    out = dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), cov2d=np.zeros((n, 3)),
               opacity=np.zeros(n), rgb=np.zeros((n, 3)), depth=np.zeros(n),
               depth_key=np.zeros(n, np.uint32), visible=np.zeros(n, np.int32),
               rect=np.zeros((n, 4), np.int32), flags=np.zeros(n, np.int32))
    lib().oracle_project(n, deg, _ptr(means), _ptr(ls), _ptr(q), _ptr(lg), _ptr(sh),
                         _ptr(camera_array(cam)), int(cam.width), int(cam.height),
                         float(near_plane), _ptr(out["mean2d"]), _ptr(out["conic"]),
                         _ptr(out["cov2d"]), _ptr(out["opacity"]), _ptr(out["rgb"]),
                         _ptr(out["depth"]), _ptr(out["depth_key"]), _ptr(out["visible"]),
                         _ptr(out["rect"]), _ptr(out["flags"]))
    if footprint not in ("ellipse", "3sigma"):
        raise ValueError("footprint must be 'ellipse' or '3sigma'")
    out["footprint"] = footprint
    out["width"], out["height"] = int(cam.width), int(cam.height)
    if footprint == "3sigma":
        footprint_3sigma(out, near_plane)
    gid, tx, ty, hit, border = footprint_tiles(out)
    out["tiles_touched"] = np.bincount(gid[hit], minlength=n).astype(np.int64)
    out["flags"] |= (np.bincount(gid[border], minlength=n) > 0).astype(np.int32)
    out["n"] = n
    return out


# ----------------------------------------------------------------------------
# Compositing (Eq. 2) and its adjoint
# ----------------------------------------------------------------------------
def all_pixels(width: int, height: int) -> np.ndarray:
    ys, xs = np.mgrid[0:height, 0:width]
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)


def render_pixels(proj: dict, pixels, bg=(0.0, 0.0, 0.0)):
    """Per pixel: colour (3), T_final, number composited, decision margin."""
    pix = _c(pixels, np.int32).reshape(-1, 2)
    m = pix.shape[0]
    color = np.zeros((m, 3))
    T = np.zeros(m)
    nc = np.zeros(m, np.int32)
    mg = np.zeros(m)
    bgd = _c(bg, np.float64)

    def run(visible, rows):
        sub = np.ascontiguousarray(pix[rows])
        c, t, k, g = np.zeros((rows.size, 3)), np.zeros(rows.size), np.zeros(rows.size, np.int32), \
            np.zeros(rows.size)
        lib().oracle_render_pixels(proj["n"], _ptr(proj["mean2d"]), _ptr(proj["conic"]),
                                   _ptr(proj["opacity"]), _ptr(proj["rgb"]), _ptr(proj["depth_key"]),
                                   _ptr(visible), rows.size, _ptr(sub), _ptr(bgd), _ptr(c),
                                   _ptr(t), _ptr(k), _ptr(g))
        color[rows], T[rows], nc[rows], mg[rows] = c, t, k, g

    if proj.get("footprint") == "3sigma":
        _tile_restricted(proj, pix, run)
    else:
        run(_c(proj["visible"], np.int32), np.arange(m))
    return color, T, nc, mg


def render_image(proj: dict, bg=(0.0, 0.0, 0.0)):
    """Full planar image [3][H][W], T_final [H][W], n_composited, margin."""
    W, H = proj["width"], proj["height"]
    color, T, nc, mg = render_pixels(proj, all_pixels(W, H), bg)
    return (color.T.reshape(3, H, W), T.reshape(H, W), nc.reshape(H, W), mg.reshape(H, W))


def render_backward_pixels(proj: dict, pixels, dL_dC, bg=(0.0, 0.0, 0.0)):
    """Gradients w.r.t. the projected quantities, (n, 9):
    [mean2d x, y, conic a, b, c, opacity, r, g, b], plus the sum of |terms|."""
    pix = _c(pixels, np.int32).reshape(-1, 2)
    g = _c(dL_dC, np.float64).reshape(-1, 3)
    assert g.shape[0] == pix.shape[0]
    n = proj["n"]
    grad = np.zeros((n, 9))
    gabs = np.zeros((n, 9))

    def run(visible, rows):
        gr, ga = np.zeros((n, 9)), np.zeros((n, 9))
        lib().oracle_render_backward_pixels(n, _ptr(proj["mean2d"]), _ptr(proj["conic"]),
                                            _ptr(proj["opacity"]), _ptr(proj["rgb"]),
                                            _ptr(proj["depth_key"]), _ptr(visible), rows.size,
                                            _ptr(np.ascontiguousarray(pix[rows])),
                                            _ptr(_c(bg, np.float64)),
                                            _ptr(np.ascontiguousarray(g[rows])), _ptr(gr), _ptr(ga))
        grad[:] += gr
        gabs[:] += ga

    if proj.get("footprint") == "3sigma":
        _tile_restricted(proj, pix, run)
    else:
        run(_c(proj["visible"], np.int32), np.arange(pix.shape[0]))
    return grad, gabs


def render_backward_image(proj: dict, dL_dimage, bg=(0.0, 0.0, 0.0)):
    W, H = proj["width"], proj["height"]
    g = np.asarray(dL_dimage, np.float64).reshape(3, H * W).T
    return render_backward_pixels(proj, all_pixels(W, H), g, bg)


def project_backward(p, cam, visible, g_proj, near_plane: float = NEAR_PLANE, grads=None,
                     stats=None):
    """Chain rule from projected-quantity gradients to raw parameters (summed
    into `grads`, so several views accumulate); optional densification
    statistic (accum, denom) accumulated in FP64."""
    n = int(p.means.shape[1])
    deg = int(p.sh_degree)
    K = (deg + 1) ** 2
    if grads is None:
        grads = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
                     opacity_logits=np.zeros(n), sh=np.zeros((K, 3, n)))
    acc = den = None
    if stats is not None:
        acc, den = stats
    lib().oracle_project_backward(
        n, deg, _ptr(_c(p.means, np.float32)), _ptr(_c(p.log_scales, np.float32)),
        _ptr(_c(p.quats, np.float32)), _ptr(_c(p.opacity_logits, np.float32)),
        _ptr(_c(p.sh, np.float32)), _ptr(camera_array(cam)), int(cam.width), int(cam.height),
        float(near_plane), _ptr(_c(visible, np.int32)), _ptr(_c(g_proj, np.float64)),
        _ptr(grads["means"]), _ptr(grads["log_scales"]), _ptr(grads["quats"]),
        _ptr(grads["opacity_logits"]), _ptr(grads["sh"]), _ptr(acc), _ptr(den))
    return grads


def l1_loss_grad(image, target):
    """L1 term of Eq. 3: mean |C - target| over 3HW, gradient sign(C - target)/(3HW)."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    return float(np.abs(d).mean()), np.sign(d) / d.size


# ----------------------------------------------------------------------------
# Tile binning by definition (the footprint rectangles, depth-ordered lists)
# ----------------------------------------------------------------------------
FOOTPRINT_INFLATE = 1.0 + 1.0 / 1024.0


def footprint_3sigma(proj: dict, near_plane: float = NEAR_PLANE):
    """The original 3DGS binning, in place on a projection: every Gaussian in
    front of the camera is binned to the tiles whose 16x16 squares meet the
    square [u - r, u + r] x [v - r, v + r], r = ceil(3 sqrt(lambda_max)) with
    lambda_max the larger eigenvalue of Sigma' (dilation included), whatever
    its opacity.  Sets visible (non-empty), rect (tiles, inclusive) and flags
    bit 0 where the radius or a square edge lies within rounding distance of
    a decision."""
    m = proj["mean2d"]
    cv = proj["cov2d"]
    d = proj["depth"]
    txn = (proj["width"] + TILE - 1) // TILE
    tyn = (proj["height"] + TILE - 1) // TILE
    with np.errstate(invalid="ignore", over="ignore"):
        front = (d > near_plane) & np.isfinite(m).all(axis=1)
        a, b, c = cv[:, 0], cv[:, 1], cv[:, 2]
        mid = 0.5 * (a + c)
        lam = mid + np.sqrt(np.maximum(mid * mid - (a * c - b * b), 0.0))
        r3 = 3.0 * np.sqrt(lam)
        r = np.ceil(r3)
        edges = [(m[:, 0] - r) / TILE, (m[:, 0] + r) / TILE, (m[:, 1] - r) / TILE, (m[:, 1] + r) / TILE]
        x0 = np.maximum(np.ceil(edges[0]) - 1, 0)
        x1 = np.minimum(np.floor(edges[1]), txn - 1)
        y0 = np.maximum(np.ceil(edges[2]) - 1, 0)
        y1 = np.minimum(np.floor(edges[3]), tyn - 1)
        vis = front & (x0 <= x1) & (y0 <= y1)

        def near_int(v):
            return np.abs(v - np.round(v)) <= 1e-6 * np.maximum(1.0, np.abs(v))
        border = near_int(r3)
        for e in edges:
            border |= near_int(e)
    rect = np.zeros((proj["n"] if "n" in proj else m.shape[0], 4), np.int32)
    rect[vis] = np.stack([x0, x1, y0, y1], axis=1)[vis].astype(np.int32)
    proj["visible"] = vis.astype(np.int32)
    proj["rect"] = rect
    proj["flags"] = (proj["flags"] & ~1) | (front & border).astype(np.int32)


def _tile_restricted(proj: dict, pix, call):
    """Under the 3-sigma footprint a pixel sees only the Gaussians binned to
    its tile: run call(visible, pixel rows) once per tile with visibility
    restricted to those Gaussians."""
    txn = (proj["width"] + TILE - 1) // TILE
    tile = (pix[:, 1] // TILE) * txn + pix[:, 0] // TILE
    r = proj["rect"]
    for t in np.unique(tile):
        tx, ty = t % txn, t // txn
        vis = proj["visible"] * ((r[:, 0] <= tx) & (tx <= r[:, 1]) & (r[:, 2] <= ty) & (ty <= r[:, 3]))
        call(np.ascontiguousarray(vis, np.int32), np.flatnonzero(tile == t))


def footprint_tiles(proj: dict):
    """The tiles a Gaussian is binned to: the tiles of its footprint rectangle
    whose 16x16 square [16 tx, 16 tx + 16] x [16 ty, 16 ty + 16] meets the ellipse
    d^T Q d <= 2 ln(255 o) (1 + 2^-10)^2 (the footprint ellipse, inflated like the
    rectangle).  Returns, for every (Gaussian, rectangle tile) pair: Gaussian id,
    tx, ty, whether the square meets the ellipse, and whether that decision lies
    within 1e-5 (relative) of flipping.  The minimum of the quadratic form over a
    square is 0 if the centre lies inside, else its minimum over the four edges
    (on an edge the minimiser of a convex quadratic is its stationary point
    clamped to the edge).  Under the 3-sigma footprint every rectangle tile is
    binned."""
    if proj.get("footprint") == "3sigma":
        vis = np.flatnonzero(proj["visible"] > 0)
        r = proj["rect"][vis].astype(np.int64)
        w = r[:, 1] - r[:, 0] + 1
        cnt = w * (r[:, 3] - r[:, 2] + 1)
        j = np.repeat(np.arange(vis.size), cnt)
        k = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        gid = vis[j]
        return (gid, r[j, 0] + k % w[j], r[j, 2] + k // w[j], np.ones(gid.size, bool),
                (proj["flags"][gid] & 1) > 0)
    vis = np.flatnonzero(proj["visible"] > 0)
    r = proj["rect"][vis].astype(np.int64)
    w = r[:, 1] - r[:, 0] + 1
    h = r[:, 3] - r[:, 2] + 1
    cnt = w * h
    j = np.repeat(np.arange(vis.size), cnt)
    k = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    tx = r[j, 0] + k % w[j]
    ty = r[j, 2] + k // w[j]
    m = proj["mean2d"][vis][j]
    a, b, c = (proj["conic"][vis][j, u] for u in range(3))
    o = proj["opacity"][vis][j]
    x0 = TILE * tx - m[:, 0]
    x1 = x0 + TILE
    y0 = TILE * ty - m[:, 1]
    y1 = y0 + TILE

    def q(x, y):
        return a * x * x + 2.0 * b * x * y + c * y * y

    inside = (x0 <= 0) & (x1 >= 0) & (y0 <= 0) & (y1 >= 0)
    qmin = np.where(inside, 0.0, np.inf)
    for X in (x0, x1):
        qmin = np.minimum(qmin, q(X, np.clip(-b * X / c, y0, y1)))
    for Y in (y0, y1):
        qmin = np.minimum(qmin, q(np.clip(-b * Y / a, x0, x1), Y))
    lim = 2.0 * np.log(255.0 * o) * FOOTPRINT_INFLATE ** 2
    hit = qmin <= lim
    border = np.abs(qmin - lim) <= 1e-5 * lim + 1e-6
    return vis[j], tx, ty, hit, border


def tile_lists(proj: dict, tile_base: int = 0):
    """Per tile of the view: the Gaussians binned to it (footprint_tiles),
    ordered by (FP32 depth bits, Gaussian index).  Returns (tile ids,
    Gaussian ids) in global order (tile, depth, index) and ranges [T, 2]."""
    W, H = proj["width"], proj["height"]
    tx_n = (W + TILE - 1) // TILE
    ty_n = (H + TILE - 1) // TILE
    gid, tx, ty, hit, _ = footprint_tiles(proj)
    gids = gid[hit]
    tiles = (ty * tx_n + tx)[hit]
    keys = proj["depth_key"][gids]
    order = np.lexsort((gids, keys, tiles))
    tiles = tiles[order] + tile_base
    gids = gids[order]
    T = tx_n * ty_n
    counts = np.bincount(tiles - tile_base, minlength=T)
    ends = np.cumsum(counts)
    ranges = np.stack([ends - counts, ends], axis=1)
    return tiles, gids, ranges


# ----------------------------------------------------------------------------
# Philox4x32-10 and split sampling
# ----------------------------------------------------------------------------
def philox4x32_10(counter, key):
    c = _c(counter, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def split_normals(seed: int, step: int, parent: int, child: int):
    z = np.zeros(3)
    w = np.zeros(4, np.uint32)
    lib().oracle_split_normals(seed, step, parent, child, _ptr(z), _ptr(w))
    return z, w


def split_means(means, log_scales, quats, parents, children, seed, step):
    n = int(means.shape[1])
    par = _c(parents, np.int64)
    ch = _c(children, np.int32)
    out = np.zeros((par.size, 3))
    lib().oracle_split_means(n, _ptr(_c(means, np.float32)), _ptr(_c(log_scales, np.float32)),
                             _ptr(_c(quats, np.float32)), par.size, _ptr(par), _ptr(ch), seed, step,
                             _ptr(out))
    return out


# ----------------------------------------------------------------------------
# Densification (Preliminary, last paragraph; global-to-local framework)
# ----------------------------------------------------------------------------
KEEP, CLONE, SPLIT0, SPLIT1 = 0, 1, 2, 3
LN_SPLIT_SHRINK = math.log(1.6)


def stats_f32(dmean2d, visible, view_wh, accum=None, denom=None):
    """Densification statistic in FP32 (the precision of the split/clone
    decision): per visible view, accum += ||g * (W/2, H/2)||, denom += 1."""
    g = _c(dmean2d, np.float32)
    V, _, n = g.shape
    acc = np.zeros(n, np.float32) if accum is None else _c(accum, np.float32).copy()
    den = np.zeros(n, np.float32) if denom is None else _c(denom, np.float32).copy()
    lib().oracle_stats_f32(n, V, _ptr(g), _ptr(_c(visible, np.int32)), _ptr(_c(view_wh, np.int32)),
                           _ptr(acc), _ptr(den))
    return acc, den


def thresholds(grad_threshold=2e-4, scale_ratio=0.01, extent=4.4, prune_opacity=0.005):
    """Raw-parameter thresholds: (tau_g, ln(rho E), logit(tau_o)) as FP32."""
    return (np.float32(grad_threshold), np.float32(math.log(scale_ratio * extent)),
            np.float32(math.log(prune_opacity / (1.0 - prune_opacity))))


# what a selected Gaussian becomes (the C oracle's mode argument)
SPLIT_LARGE, ADAPTIVE, SPLIT_ONLY, CLONE_ONLY = 0, 1, 2, 3


def select(accum, denom, log_scales, logits, tau_g, log_scale_thr, logit_thr, mode=ADAPTIVE):
    """Split / clone / prune masks; mode SPLIT_LARGE (global phase), ADAPTIVE
    (3DGS rule), SPLIT_ONLY or CLONE_ONLY (the single-operation variants).  A
    bool mode reads as clones allowed (True = ADAPTIVE, False = SPLIT_LARGE)."""
    if int(mode) not in (SPLIT_LARGE, ADAPTIVE, SPLIT_ONLY, CLONE_ONLY):
        raise ValueError("unknown densification mode %r" % (mode,))
    n = int(np.asarray(accum).size)
    s = np.zeros(n, np.uint8)
    c = np.zeros(n, np.uint8)
    p = np.zeros(n, np.uint8)
    lib().oracle_select(n, _ptr(_c(accum, np.float32)), _ptr(_c(denom, np.float32)),
                        _ptr(_c(log_scales, np.float32)), _ptr(_c(logits, np.float32)),
                        float(tau_g), float(log_scale_thr), float(logit_thr), int(mode),
                        _ptr(s), _ptr(c), _ptr(p))
    return s, c, p


def densify_plan(split, clone, prune):
    """Index map of the compaction: parent i emits nothing if pruned, else
    [SPLIT0, SPLIT1] if split, [KEEP, CLONE] if cloned, [KEEP] otherwise;
    outputs are in parent order."""
    split = np.asarray(split).astype(bool)
    clone = np.asarray(clone).astype(bool)
    prune = np.asarray(prune).astype(bool)
    counts = np.where(prune, 0, np.where(split | clone, 2, 1))
    src = np.repeat(np.arange(split.size, dtype=np.int64), counts)
    first = np.ones(src.size, bool)
    first[1:] = src[1:] != src[:-1]
    kind = np.full(src.size, KEEP, np.uint8)
    s = split[src]
    c = clone[src] & ~s
    kind[s & first] = SPLIT0
    kind[s & ~first] = SPLIT1
    kind[c & ~first] = CLONE
    return src.astype(np.int32), kind


def densify_apply(params: dict, src, kind, seed: int, step: int):
    """New parameter set (FP64): split children get mu + R(s * z) and
    log-scale - ln 1.6; clones and kept rows copy the parent."""
    src = np.asarray(src, np.int64)
    kind = np.asarray(kind)
    out = {}
    for name, arr in params.items():
        a = np.asarray(arr, np.float64)
        out[name] = a[..., src].copy()
    sp = np.nonzero((kind == SPLIT0) | (kind == SPLIT1))[0]
    if sp.size:
        child = (kind[sp] == SPLIT1).astype(np.int32)
        mu = split_means(params["means"], params["log_scales"], params["quats"], src[sp], child,
                         seed, step)
        out["means"][:, sp] = mu.T
        out["log_scales"][:, sp] = np.asarray(params["log_scales"], np.float64)[:, src[sp]] - \
            LN_SPLIT_SHRINK
    return out


def morton_code(qx: int, qy: int, qz: int) -> int:
    """Interleave three 10-bit cell coordinates bit by bit: bit b of qx goes to
    bit 3b, of qy to 3b + 1, of qz to 3b + 2."""
    code = 0
    for b in range(10):
        code |= ((qx >> b) & 1) << (3 * b)
        code |= ((qy >> b) & 1) << (3 * b + 1)
        code |= ((qz >> b) & 1) << (3 * b + 2)
    return code


def spatial_order(means):
    """The Morton-order permutation of Gaussians (a memory layout, not a step
    of the paper's method): cells of a 1024^3 grid over the cube of the finite
    means' bounding box (side = longest extent), q = min(1023, trunc((x - lo) *
    (1024 / side))) evaluated in FP32 (the precision the layout is decided in),
    non-finite means last, ties by index.  Returns (src, codes)."""
    m = np.asarray(means, np.float32)
    n = m.shape[1]
    fin = np.isfinite(m).all(axis=0)
    codes = np.full(n, 0x3FFFFFFF, np.int64)
    if fin.any():
        lo = m[:, fin].min(axis=1)
        hi = m[:, fin].max(axis=1)
        side = np.float32(max(np.float32(hi[a] - lo[a]) for a in range(3)))
        inv = np.float32(np.float32(1024.0) / side) if side > 0 else np.float32(0.0)
        for i in np.flatnonzero(fin):
            q = []
            for a in range(3):
                t = np.float32(np.float32(m[a, i] - lo[a]) * inv)
                q.append(1023 if t >= np.float32(1023.0) else int(t))
            codes[i] = morton_code(*q)
    src = np.argsort(codes, kind="stable").astype(np.int32)
    return src, codes


def lineage_apply(origin, splits, clones, src, kind):
    """Lineage attributes through one densification (Methodology, Spatial
    diffusion): every output row keeps its parent's original position; both
    children of a split count one more split than the parent, and both copies
    of a cloned parent (the kept one and the clone, which are identical) one
    more clone.  FP64."""
    src = np.asarray(src, np.int64)
    kind = np.asarray(kind)
    o = np.asarray(origin, np.float64)[..., src].copy()
    s = np.asarray(splits, np.float64)[..., src] + ((kind == SPLIT0) | (kind == SPLIT1))
    cloned_parents = np.unique(src[kind == CLONE])
    c = np.asarray(clones, np.float64)[..., src] + np.isin(src, cloned_parents)
    return o, s, c


def lineage_categories(splits, clones):
    """Split-dominated (splits > clones) = 0, clone-dominated = 1, equal = 2."""
    s = np.asarray(splits)
    c = np.asarray(clones)
    return np.where(s > c, 0, np.where(c > s, 1, 2)).astype(np.int8)


def adaptive_prune_logit(logits, p=0.03, tau_u=0.05):
    """Adaptive opacity threshold (Methodology, Adaptive Opacity Pruning):
    tau = min(alpha_sorted[floor(N p)], tau_u), returned in logit space
    (sigmoid is monotone, so alpha < tau  <=>  logit < logit(tau))."""
    lg = np.sort(np.asarray(logits, np.float32), kind="stable")
    k = int(math.floor(lg.size * p))
    k = min(k, lg.size - 1)
    upper = np.float32(math.log(tau_u / (1.0 - tau_u)))
    return np.float32(min(lg[k], upper)), k


# ----------------------------------------------------------------------------
# Sparse Adam (the optimiser of the accelerated training the paper builds on)
# ----------------------------------------------------------------------------
def adam_step(param, grad, m, v, lr, visible, beta1, beta2, eps, step):
    """One sparse Adam step in FP64 on arrays [..., n]: the columns i with
    visible[i] take m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2 and
    p -= lr m_hat / (sqrt(v_hat) + eps) with m_hat = m / (1 - b1^step),
    v_hat = v / (1 - b2^step); the other columns are returned unchanged."""
    p = np.array(param, np.float64)
    g = np.asarray(grad, np.float64)
    m = np.array(m, np.float64)
    v = np.array(v, np.float64)
    sel = np.asarray(visible, bool)
    m2 = beta1 * m + (1 - beta1) * g
    v2 = beta2 * v + (1 - beta2) * g * g
    mh = m2 / (1 - beta1 ** step)
    vh = v2 / (1 - beta2 ** step)
    p2 = p - lr * mh / (np.sqrt(vh) + eps)
    p[..., sel] = p2[..., sel]
    m[..., sel] = m2[..., sel]
    v[..., sel] = v2[..., sel]
    return p, m, v
