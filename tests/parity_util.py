"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same seeded inputs, and compare."""
import json
import math
import os

import numpy as np
import torch

import oracle
from paper_2507_20239_amd import gsmi

MARGIN = 1e-5      # decisions closer than this (relative) to a threshold are excluded
RTOL = 1e-4        # FP32 vs FP64 bound for images and gradients


def dev():
    return torch.device("cuda:0")


def params_of(sc, device=None):
    device = device or dev()
    return {k: torch.from_numpy(np.ascontiguousarray(getattr(sc, k))).to(device)
            for k in gsmi.PARAM_NAMES}


def gpu_forward(sc, cams, opts=None, cap=1 << 22, frame=None):
    """Project + render every camera in one frame.  Returns (frame, images list)."""
    opts = opts or gsmi.raster_opts(bg=tuple(float(x) for x in sc.bg), count_composited=True)
    params = params_of(sc)
    cams_dev = gsmi.cameras_to_device(cams, dev())
    if frame is None:
        frame = gsmi.Frame(sc.n, [(c.width, c.height) for c in cams], cap, dev())
    frame.project(params, sc.sh_degree, cams_dev, opts)
    flat = frame.render(opts)
    torch.cuda.synchronize()
    return frame, flat, params, cams_dev, opts


def splat_view(frame):
    """(E, 12) float32 numpy copy of the projected splats."""
    return frame.buffer(gsmi.BUF_SPLAT, torch.float32).view(-1, 12).cpu().numpy()


KAPPA = math.log2(math.e) / 2


def oracle_chol(conic):
    """Cholesky factor (l11, l21, l22) of kappa * conic, the form the splat
    record stores (kappa = log2(e)/2), from the oracle's FP64 conic."""
    a, b, c = np.asarray(conic, np.float64).T
    l11 = np.sqrt(KAPPA * a)
    return np.stack([l11, KAPPA * b / l11, np.sqrt(KAPPA * (c - b * b / a))], 1)


def check_chol(got, conic, rtol=1e-5, what="conic factor"):
    """The stored factor against the oracle's; l21 is measured against
    sqrt(l21^2 + l22^2) = sqrt(kappa c), the scale its rounding error has."""
    ref = oracle_chol(conic)
    scale = np.stack([ref[:, 0], np.hypot(ref[:, 1], ref[:, 2]), ref[:, 2]], 1)
    assert_close_scaled(got, ref, scale, rtol=rtol, what=what)


def gpu_mean2d(sp):
    return sp[:, 0:2].astype(np.float64) + sp[:, 2:4].astype(np.float64)


def raw_grad_scale(sc, cam, p, gabs):
    """Upper bound of sum_p |per-pixel raw-parameter gradient term| per element:
    |J_i| applied to the oracle's per-splat absolute term sums (J_i = Jacobian of
    the nine projected quantities w.r.t. the raw parameters of Gaussian i)."""
    n = sc.n
    K = (sc.sh_degree + 1) ** 2
    out = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
               opacity_logits=np.zeros(n), sh=np.zeros((K, 3, n)))
    # only Gaussians that received gradient terms contribute
    vis = np.asarray(p["visible"], np.int32) * (np.asarray(gabs) > 0).any(1)
    for k in range(9):
        g = np.zeros((n, 9))
        g[:, k] = 1.0
        J = oracle.project_backward(sc, cam, vis, g)
        for name in out:
            out[name] += np.abs(J[name]) * gabs[:, k]
    return out


def _report(what, **vals):
    """Append one line per comparison to $GSMI_PARITY_REPORT (JSON lines), so
    a run can list how close every suite came to its bars."""
    path = os.environ.get("GSMI_PARITY_REPORT")
    if not path:
        return
    rec = {"test": os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0], "what": what}
    rec.update({k: (float(v) if v is not None else None) for k, v in vals.items()})
    with open(path, "a") as fh:
        fh.write(json.dumps(rec) + "\n")


def assert_close_scaled(got, ref, scale, rtol=RTOL, what=""):
    """FP32 result against the FP64 oracle, both bars of the parity metric:
    elementwise |x - x64| <= rtol max(|x64|, a64), with a64 the oracle's
    magnitude scale of the element (the sum of the magnitudes of the terms a
    gradient is made of, |C| + |bg| for a pixel), and norm-wise
    ||x - x64||_2 <= rtol ||x64||_2 over the whole array."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.broadcast_to(np.asarray(scale, np.float64), ref.shape)
    tol = rtol * np.maximum(np.abs(ref), scale) + 1e-30
    err = np.abs(got - ref)
    bad = err > tol
    nrm = float(np.linalg.norm(ref))
    enrm = float(np.linalg.norm(got - ref))
    _report(what, n=ref.size, norm_ratio=enrm / nrm if nrm > 0 else None,
            elem_ratio=float((err / tol).max()) * rtol if err.size else 0.0)
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError("%s: %d/%d elements outside tolerance, e.g. %s got %s ref %s scale %s"
                             % (what, int(bad.sum()), bad.size, idx.tolist(),
                                got[bad][:5], ref[bad][:5], scale[bad][:5]))
    if nrm > 0:
        assert enrm <= rtol * nrm, "%s: ||x - x64|| / ||x64|| = %.3g > %g" % (what, enrm / nrm, rtol)
    else:
        assert enrm <= rtol * float(np.linalg.norm(scale)) + 1e-30, what


def _norm_ranges(r):
    """Ranges with empty tiles written as [0, 0] (the GPU leaves them zero)."""
    r = np.asarray(r, np.int64).copy()
    r[r[:, 0] == r[:, 1]] = 0
    return r


def _check_ranges_partition(gr, gt):
    """Ranges are the runs of equal tile ids of the sorted instance list."""
    n = gt.size
    starts = np.flatnonzero(np.r_[True, gt[1:] != gt[:-1]]) if n else np.zeros(0, np.int64)
    ends = np.r_[starts[1:], n] if n else starts
    want = np.zeros_like(gr, dtype=np.int64)
    want[gt[starts], 0] = starts
    want[gt[starts], 1] = ends
    np.testing.assert_array_equal(_norm_ranges(gr), _norm_ranges(want))


def _compare_lists(p, gt, ge, tiles, gids, entry_base=0):
    """Bit-exact (tile, Gaussian) order, leaving out the Gaussians whose footprint
    rectangle lies within 1e-3 px of a tile-edge decision (reported by the oracle)."""
    flagged = np.flatnonzero(p["flags"] & 1)
    assert flagged.size <= max(2, p["n"] // 500)
    kg = ~np.isin(ge - entry_base, flagged)
    ko = ~np.isin(gids, flagged)
    np.testing.assert_array_equal(gt[kg], tiles[ko])
    np.testing.assert_array_equal(ge[kg] - entry_base, gids[ko])
    return flagged.size
