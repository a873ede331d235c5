"""The torch.autograd path (GaussianRasterizer): gradients against the
oracle's analytic adjoint on small multi-view scenes, against central finite
differences of the FP64 oracle on a 64-Gaussian slice of the 6,000,000-Gaussian
procedural scene (4 views of 1920x1080), the densification statistic as a side
effect of the backward, instance-capacity growth, and the guard against a
backward whose frame was overwritten."""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_2507_20239_amd import gsmi, synth
from paper_2507_20239_amd.autograd import GaussianRasterizer
from parity_util import MARGIN, _report, assert_close_scaled, dev, raw_grad_scale

pytestmark = pytest.mark.gpu


def _leaf_params(sc):
    return {k: torch.from_numpy(np.ascontiguousarray(getattr(sc, k))).to(dev()).requires_grad_()
            for k in gsmi.PARAM_NAMES}


def _call(r, P):
    return r(P["means"], P["log_scales"], P["quats"], P["opacity_logits"], P["sh"])


def _subscene(sc, idx):
    idx = np.sort(np.asarray(idx))
    return synth.Scene(sc.means[:, idx].copy(), sc.log_scales[:, idx].copy(),
                       sc.quats[:, idx].copy(), sc.opacity_logits[idx].copy(),
                       sc.sh[:, :, idx].copy(), sc.sh_degree, [], [], sc.bg), idx


def test_autograd_gradients_match_oracle_adjoint():
    sc = synth.random_scene(51, 800, 96, 80, sh_degree=3, n_views=2, log_scale=(-2.5, 0.5))
    cams = [sc.cameras[0], sc.cameras[1].scaled(2)]
    r = GaussianRasterizer(sc.n, cams, sc.sh_degree, device=dev())
    P = _leaf_params(sc)
    imgs = _call(r, P)
    rng = np.random.default_rng(3)
    Ws, projs = [], []
    for cam in cams:
        p = oracle.project(sc, cam)
        _, _, _, margin = oracle.render_image(p)
        w = rng.standard_normal((3, cam.height, cam.width)) * 1e-2
        w[:, margin <= MARGIN] = 0.0
        Ws.append(w.astype(np.float32))
        projs.append(p)
    loss = sum((img * torch.from_numpy(w).to(dev())).sum() for img, w in zip(imgs, Ws))
    loss.backward()
    want = {k: 0.0 for k in gsmi.PARAM_NAMES}
    scale = {k: 0.0 for k in gsmi.PARAM_NAMES}
    den = np.zeros(sc.n)
    for cam, p, w in zip(cams, projs, Ws):
        gproj, gabs = oracle.render_backward_image(p, w.astype(np.float64))
        acc, dn = np.zeros(sc.n), np.zeros(sc.n)
        g = oracle.project_backward(sc, cam, p["visible"], gproj, stats=(acc, dn))
        s = raw_grad_scale(sc, cam, p, gabs)
        for k in gsmi.PARAM_NAMES:
            want[k] = want[k] + g[k]
            scale[k] = scale[k] + s[k]
        den += dn
    for k in gsmi.PARAM_NAMES:
        assert_close_scaled(P[k].grad.cpu().numpy(), want[k], scale[k], what=k)
    # the statistic's count: views in which each Gaussian was rendered
    np.testing.assert_array_equal(r.denom.cpu().numpy(), den)


def test_autotuned_rasterizer_matches_the_default_shape(tmp_path, monkeypatch):
    """autotune=True picks a launch shape on the first call; the images are
    the same bit for bit and the gradients agree to FP32 summation order."""
    monkeypatch.setenv("GSMI_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    sc = synth.random_scene(52, 3000, 96, 80, sh_degree=2, n_views=3, log_scale=(-2.3, 0.5))
    cams = [sc.cameras[0], sc.cameras[1].scaled(2), sc.cameras[2]]
    out = []
    for tune in (False, True):
        r = GaussianRasterizer(sc.n, cams, sc.sh_degree, device=dev(), autotune=tune)
        P = _leaf_params(sc)
        imgs = _call(r, P)
        loss = sum((img * (k + 1.0)).sum() for k, img in enumerate(imgs))
        loss.backward()
        out.append(([i.detach().clone() for i in imgs], {k: P[k].grad.clone() for k in P}))
        if tune:
            assert r.tuned is not None and r.tuned["candidates"] >= 4
            assert (tmp_path / "tune.json").exists()
    for a, b in zip(out[0][0], out[1][0]):
        assert torch.equal(a, b)
    for k in gsmi.PARAM_NAMES:
        a, b = out[0][1][k], out[1][1][k]
        assert torch.allclose(a, b, rtol=1e-4, atol=1e-6 * float(a.abs().max())), k


def test_capacity_grows_and_images_do_not_change():
    sc = synth.random_scene(52, 1500, 128, 96, sh_degree=1, log_scale=(-2.0, 0.5))
    P = _leaf_params(sc)
    small = GaussianRasterizer(sc.n, sc.cameras, sc.sh_degree, device=dev(), capacity=256)
    big = GaussianRasterizer(sc.n, sc.cameras, sc.sh_degree, device=dev(), capacity=1 << 20)
    a = _call(small, P)[0]
    b = _call(big, P)[0]
    assert small.frame.cap > 256
    assert torch.equal(a, b)


def test_stale_backward_raises():
    sc = synth.random_scene(53, 300, 64, 48, sh_degree=0)
    P = _leaf_params(sc)
    r = GaussianRasterizer(sc.n, sc.cameras, sc.sh_degree, device=dev())
    first = _call(r, P)[0].sum()
    _call(r, P)
    with pytest.raises(RuntimeError, match="rendered again"):
        first.backward()


# ---------------------------------------------------------------------------
# 6,000,000 Gaussians on spheres and planes, 4 views of 1920x1080
# ---------------------------------------------------------------------------
def _rect_pixels(rect, W, H):
    x0, x1, y0, y1 = (int(v) for v in rect)
    ys, xs = np.mgrid[y0 * 16:min((y1 + 1) * 16, H), x0 * 16:min((x1 + 1) * 16, W)]
    return np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)


def _overlapping(p, tiles, tiles_x, tiles_y, among=None):
    """Gaussians (among `among`, default all visible) whose footprint rectangle
    meets any tile of `tiles` ([m, 2] of (tx, ty)): a summed-area table of the
    tile mask, evaluated per rectangle."""
    m = np.zeros((tiles_y + 1, tiles_x + 1), np.int64)
    m[tiles[:, 1] + 1, tiles[:, 0] + 1] = 1
    sat = m.cumsum(0).cumsum(1)
    vis = np.flatnonzero(p["visible"] > 0) if among is None else among
    x0, x1, y0, y1 = (p["rect"][vis, k] for k in range(4))
    cnt = sat[y1 + 1, x1 + 1] - sat[y0, x1 + 1] - sat[y1 + 1, x0] + sat[y0, x0]
    return vis[cnt > 0]


def _support_tiles(items):
    return sorted({tuple(t) for _, rect, _ in items for t in _tiles_of(rect)})


def _tiles_of(rect):
    x0, x1, y0, y1 = (int(v) for v in rect)
    ty, tx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
    return np.stack([tx.ravel(), ty.ravel()], 1)


@pytest.fixture(scope="module")
def scene_6m_1920x1080():
    sc = synth.procedural_scene()
    cams = synth.procedural_cameras()[:4]
    sc.cameras = cams
    projs = [oracle.project(sc, cam) for cam in cams]
    return sc, cams, projs


def _tile_pixels(tx, ty, W, H):
    return _rect_pixels((tx, tx, ty, ty), W, H)


def c5_slice_and_weights(sc, cams, projs, seed=9, m=64):
    """64 Gaussians rendered in view 0 inside a single tile with no flagged
    decision, and loss weights: random on every tile they cover in any view,
    zero on pixels where a compositing decision lies within rounding distance
    of its threshold."""
    rng = np.random.default_rng(seed)
    p0 = projs[0]
    r0 = p0["rect"]
    single = np.flatnonzero((p0["visible"] > 0) & (p0["flags"] == 0) & (r0[:, 0] == r0[:, 1]) &
                            (r0[:, 2] == r0[:, 3]))
    assert single.size > 10 * m
    slice_ids = np.sort(rng.choice(single, m, replace=False))
    Ws = [np.zeros((3, c.height, c.width), np.float32) for c in cams]
    support = []   # per view: list of (gaussian, rect, pixels)
    for v, (cam, p) in enumerate(zip(cams, projs)):
        items = []
        for g in slice_ids:
            if p["visible"][g] > 0:
                items.append((g, p["rect"][g].copy(),
                               _rect_pixels(p["rect"][g], cam.width, cam.height)))
        support.append(items)
        tiles = _support_tiles(items)
        if not tiles:
            continue
        txy = ((cam.width + 15) // 16, (cam.height + 15) // 16)
        cand = _overlapping(p, np.array(tiles), *txy)
        for tx, ty in tiles:
            pix = _tile_pixels(tx, ty, cam.width, cam.height)
            sub, _ = _subscene(sc, _overlapping(p, np.array([[tx, ty]]), *txy, among=cand))
            _, _, _, margin = oracle.render_pixels(oracle.project(sub, cam), pix)
            w = rng.standard_normal((3, pix.shape[0])) * 1e-2
            w[:, margin <= MARGIN] = 0.0
            Ws[v][:, pix[:, 1], pix[:, 0]] = w
    return slice_ids, Ws, support


def oracle_slice_grads(sc, cams, projs, Ws, support, slice_ids):
    """The oracle's analytic raw-parameter gradients of sum_v W_v . image_v for
    the slice and their error scales, tile by tile over the weighted tiles with
    the Gaussians that reach each tile."""
    want = {k: np.zeros(getattr(sc, k).shape[:-1] + (slice_ids.size,)) for k in gsmi.PARAM_NAMES}
    scale = {k: np.zeros_like(want[k]) for k in gsmi.PARAM_NAMES}
    sl, _ = _subscene(sc, slice_ids)
    for v, (cam, p) in enumerate(zip(cams, projs)):
        gproj = np.zeros((slice_ids.size, 9))
        gabs = np.zeros((slice_ids.size, 9))
        tiles = _support_tiles(support[v])
        if not tiles:
            continue
        txy = ((cam.width + 15) // 16, (cam.height + 15) // 16)
        cand = _overlapping(p, np.array(tiles), *txy)
        for tx, ty in tiles:
            pix = _tile_pixels(tx, ty, cam.width, cam.height)
            idx = _overlapping(p, np.array([[tx, ty]]), *txy, among=cand)
            sub, idx = _subscene(sc, idx)
            ps = oracle.project(sub, cam)
            wv = Ws[v][:, pix[:, 1], pix[:, 0]].T.astype(np.float64)
            gp, ga = oracle.render_backward_pixels(ps, pix, wv)
            pos = np.searchsorted(idx, slice_ids)
            inside = (pos < idx.size) & (idx[np.minimum(pos, idx.size - 1)] == slice_ids)
            gproj[inside] += gp[pos[inside]]
            gabs[inside] += ga[pos[inside]]
        psl = oracle.project(sl, cam)
        g = oracle.project_backward(sl, cam, psl["visible"], gproj)
        s = raw_grad_scale(sl, cam, psl, gabs)
        for k in gsmi.PARAM_NAMES:
            want[k] += g[k]
            scale[k] += s[k]
    return want, scale


class FiniteDifferences:
    """Central differences of the FP64 oracle's sum_v W_v . image_v w.r.t. the 59
    raw parameters of Gaussian gid (order: means, log-scales, quats, logit, SH).
    Only the pixels inside the Gaussian's footprint can change, so only they are
    rendered, with the Gaussians that reach its tiles; a step re-projects the
    one perturbed Gaussian.  Parameters are FP32, so the step actually taken is
    the difference of the two rounded values."""

    def __init__(self, sc, cams, projs, Ws, support, gid):
        self.views = []
        for v, (cam, p) in enumerate(zip(cams, projs)):
            for (g2, rect, rp) in support[v]:
                if g2 != gid:
                    continue
                idx = _overlapping(p, _tiles_of(rect), (cam.width + 15) // 16,
                                   (cam.height + 15) // 16)
                sub, idx = _subscene(sc, idx)
                jj = int(np.searchsorted(idx, gid))
                ps = oracle.project(sub, cam)
                # pixels of the footprint {o G >= 1/255}, widened by 1%
                d = rp + 0.5 - ps["mean2d"][jj]
                a, b, c = ps["conic"][jj]
                q = a * d[:, 0] ** 2 + 2 * b * d[:, 0] * d[:, 1] + c * d[:, 1] ** 2
                lim = 2.0 * np.log(255.0 * ps["opacity"][jj]) * 1.01
                pix = rp[q <= lim]
                w = Ws[v][:, pix[:, 1], pix[:, 0]].T.astype(np.float64)
                if not w.any():
                    continue
                # keep the Gaussians whose footprint box meets these pixels' box
                o = np.maximum(ps["opacity"], 1.0 / 255.0)
                L = 2.0 * np.log(255.0 * o) * 1.01
                ex = np.sqrt(L * ps["cov2d"][:, 0]) + 1.0
                ey = np.sqrt(L * ps["cov2d"][:, 2]) + 1.0
                m2 = ps["mean2d"]
                lo, hi = pix.min(0) + 0.5, pix.max(0) + 0.5
                keep = ((ps["visible"] > 0) & (m2[:, 0] + ex >= lo[0]) & (m2[:, 0] - ex <= hi[0]) &
                        (m2[:, 1] + ey >= lo[1]) & (m2[:, 1] - ey <= hi[1]))
                keep[jj] = True
                sub, kept = _subscene(sub, np.flatnonzero(keep))
                jj = int(np.searchsorted(kept, jj))
                ps = oracle.project(sub, cam)
                one, _ = _subscene(sub, [jj])
                self.views.append((cam, sub, jj, ps, one, pix, w))
        self.slots = [(name, row) for name in gsmi.PARAM_NAMES
                      for row in range(int(np.prod(getattr(sc, name).shape[:-1])))]

    def __call__(self, k, rel_step=1e-6):
        # per-pixel differences first: summing the loss before differencing would
        # leave its own rounding (1e-16 of the whole loss) in every derivative
        name, row = self.slots[k]
        total, step = 0.0, None
        for cam, sub, jj, ps, one, pix, w in self.views:
            if pix.shape[0] == 0:
                continue
            arr = getattr(one, name)
            flat = arr.reshape(-1, 1)
            x0 = float(flat[row, 0])
            C, xs = [], []
            for sign in (-1.0, 1.0):
                x = np.float32(x0 + sign * rel_step * max(1.0, abs(x0)))
                flat[row, 0] = x
                q1 = oracle.project(one, cam)
                pp = dict(ps)
                for key in ("mean2d", "conic", "opacity", "rgb", "depth_key", "visible"):
                    pp[key] = ps[key].copy()
                    pp[key][jj] = q1[key][0]
                C.append(oracle.render_pixels(pp, pix)[0])
                xs.append(float(x))
            flat[row, 0] = np.float32(x0)
            total += float((w * (C[1] - C[0])).sum())
            step = xs[1] - xs[0]
        return total / step if step else 0.0


GROUPS = ((0, 3), (3, 6), (6, 10), (10, 11), (11, 59))
FD_RTOL = 1e-4


def check_fd(gg, want, fdiff, gid):
    """GPU gradient (FP32) against central differences of the FP64 oracle, per
    parameter group: within 1e-4 of the group's largest derivative plus 1e-4
    relative.  Where a component misses that bar and the oracle's own analytic
    gradient (FP64) misses it too, the differences are what is off: the loss is
    not smooth within the step there (the depth key is the FP32 rounding of
    the depth, a step function, so moving a mean can swap two splats of equal
    key; a pixel's alpha can cross the 1/255 cut-off).  Such a component
    counts as FD-limited if the GPU still agrees with the analytic gradient
    to 1e-4 of the group scale.  Returns (number FD-limited, largest GPU-vs-FD
    ratio per group)."""
    fd = np.array([fdiff(k) for k in range(gg.size)])
    limited = 0
    ratios = []
    for a, b in GROUPS:
        big = np.abs(fd[a:b]).max()
        r = float(np.abs(gg[a:b] - fd[a:b]).max() / big) if big > 0 else 0.0
        ra = float(np.abs(want[a:b] - fd[a:b]).max() / big) if big > 0 else 0.0
        _report("FD group %d..%d of Gaussian %d" % (a, b, gid), n=b - a, group_ratio=r,
                oracle_group_ratio=ra)
        ratios.append(r)
        for k in range(a, b):
            tol = FD_RTOL * big + FD_RTOL * abs(fd[k]) + 1e-11
            if abs(gg[k] - fd[k]) <= tol:
                continue
            assert abs(want[k] - fd[k]) > tol, (gid, k, gg[k], want[k], fd[k])
            assert abs(gg[k] - want[k]) <= FD_RTOL * max(big, abs(want[k])) + 1e-11, \
                (gid, k, gg[k], want[k], fd[k])
            limited += 1
    return limited, ratios


@pytest.fixture(scope="module")
def slice_grads(scene_6m_1920x1080, tmp_path_factory):
    """GPU autograd over the whole scene with the slice's loss weights, in the
    autotuned launch shape the benchmark times."""
    sc, cams, projs = scene_6m_1920x1080
    slice_ids, Ws, support = c5_slice_and_weights(sc, cams, projs)
    old = os.environ.get("GSMI_AUTOTUNE_CACHE")
    os.environ["GSMI_AUTOTUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "tune.json")
    try:
        r = GaussianRasterizer(sc.n, cams, sc.sh_degree, device=dev(), autotune=True)
        P = _leaf_params(sc)
        imgs = _call(r, P)
    finally:
        if old is None:
            os.environ.pop("GSMI_AUTOTUNE_CACHE", None)
        else:
            os.environ["GSMI_AUTOTUNE_CACHE"] = old
    print("tuned", r.tuned, flush=True)
    loss = sum((img * torch.from_numpy(w).to(dev())).sum() for img, w in zip(imgs, Ws))
    loss.backward()
    got = {k: P[k].grad.cpu().numpy()[..., slice_ids] for k in gsmi.PARAM_NAMES}
    assert r.frame.status()[2] == 0
    del r, P, imgs, loss
    return slice_ids, Ws, support, got


@pytest.fixture(scope="module")
def slice_oracle(scene_6m_1920x1080, slice_grads):
    sc, cams, projs = scene_6m_1920x1080
    slice_ids, Ws, support, _ = slice_grads
    return oracle_slice_grads(sc, cams, projs, Ws, support, slice_ids)


def test_6m_slice_gradients_match_oracle_adjoint(slice_grads, slice_oracle):
    got = slice_grads[3]
    want, scale = slice_oracle
    for k in gsmi.PARAM_NAMES:
        assert_close_scaled(got[k], want[k], scale[k], what="6M-Gaussian slice " + k)


@pytest.mark.parametrize("part", range(4))
def test_6m_slice_gradients_match_finite_differences(scene_6m_1920x1080, slice_grads,
                                                     slice_oracle, part):
    """Central differences on all 64 Gaussians of the slice (16 per part), all
    59 raw parameters each, at 1e-4 of the group scale."""
    sc, cams, projs = scene_6m_1920x1080
    slice_ids, Ws, support, got = slice_grads
    want = slice_oracle[0]
    limited = 0
    worst = np.zeros(len(GROUPS))
    for j in range(16 * part, 16 * part + 16):
        gid = slice_ids[j]
        fdiff = FiniteDifferences(sc, cams, projs, Ws, support, gid)
        gg = np.concatenate([got[k][..., j].reshape(-1) for k in gsmi.PARAM_NAMES])
        ww = np.concatenate([want[k][..., j].reshape(-1) for k in gsmi.PARAM_NAMES])
        n_lim, ratios = check_fd(gg, ww, fdiff, gid)
        limited += n_lim
        worst = np.maximum(worst, ratios)
    print("FD part %d: largest GPU-vs-FD ratio per group %s, FD-limited components %d"
          % (part, np.array2string(worst, precision=2), limited), flush=True)
    assert limited <= 0.02 * 16 * 59


def test_fused_adam_in_the_backward():
    """fuse_adam: the backward updates the parameter leaves in place and gives
    them no gradient; the result equals the separate projection adjoint
    followed by sparse Adam on the same frame state, bit for bit, for all five
    arrays and for the colour coefficients alone (the other four then get
    their usual gradients); the device counter is read, not advanced."""
    sc = synth.random_scene(62, 2000, 96, 80, sh_degree=3, n_views=2, log_scale=(-2.4, 0.5))
    cams = list(sc.cameras)
    names = gsmi.PARAM_NAMES
    lrs = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    for fused in (names, ("sh",)):
        P = _leaf_params(sc)
        r = GaussianRasterizer(sc.n, cams, sc.sh_degree, device=dev())
        mom = {k: (torch.zeros_like(P[k]), torch.zeros_like(P[k])) for k in fused}
        counter = gsmi.adam_counter(dev())
        counter[0] = 2
        r.fuse_adam(gsmi.FusedAdamStep(mom, lrs, counter))
        start = {k: P[k].detach().clone() for k in names}
        g = torch.Generator(device=dev())
        g.manual_seed(11)
        imgs = _call(r, P)
        loss = sum((im * torch.rand(im.shape, device=dev(), generator=g)).sum() for im in imgs)
        loss.backward()
        torch.cuda.synchronize()
        assert int(counter[0]) == 2
        grads = gsmi.empty_grads(start)
        r.frame.project_backward(start, sc.sh_degree, r.cams_dev, r.opts, grads)
        ref = {k: (start[k].clone(), torch.zeros_like(start[k]), torch.zeros_like(start[k]))
               for k in fused}
        c2 = gsmi.adam_counter(dev())
        c2[0] = 2
        gsmi.adam_step([(ref[k][0], grads[k], ref[k][1], ref[k][2], lrs[k]) for k in fused], sc.n,
                       c2, tiles_touched=r.frame.buffer(gsmi.BUF_TILES_TOUCHED), n_views=2)
        torch.cuda.synchronize()
        for k in names:
            if k in fused:
                assert P[k].grad is None, k
                assert not torch.equal(P[k].detach(), start[k]), k
                assert torch.equal(P[k].detach(), ref[k][0]), k
                assert torch.equal(mom[k][0], ref[k][1]) and torch.equal(mom[k][1], ref[k][2]), k
            else:
                assert torch.equal(P[k].detach(), start[k]), k
                assert torch.equal(P[k].grad, grads[k]), k
        r.fuse_adam(None)
        assert r.adam is None


def test_captured_training_step_replays_match_eager():
    """The whole training step (rasterize, Eq. 3 loss, backward, sparse Adam)
    captured once in a graph and replayed step after step with new views: the
    rasterizer checks its capacity lazily, takes its cameras from a device
    table row copy, and Adam counts its steps on the device.  Each replay is
    checked against the same step run eagerly from the same parameters and
    moments on a second rasterizer: the loss and the gradients (FP32 atomics,
    so to 1e-5 of their scale), and the new parameters and moments bit for bit
    against the host-counted Adam applied to the replay's own gradients."""
    from paper_2507_20239_amd.autograd import photometric_loss
    sc = synth.random_scene(61, 3000, 96, 80, sh_degree=3, n_views=4, log_scale=(-2.4, 0.5))
    cams = list(sc.cameras)
    table = gsmi.cameras_to_device(cams, dev()).view(len(cams), -1)
    pick = torch.tensor([0, 1], dtype=torch.int64, device=dev())
    cam_static = table.index_select(0, pick).reshape(-1).clone()
    r = GaussianRasterizer(sc.n, cams[:2], sc.sh_degree, device=dev(), lazy_overflow=True)
    r.use_device_cameras(cam_static)
    g = torch.Generator(device=dev())
    g.manual_seed(4)
    targets = torch.rand(len(cams), 3, 80, 96, device=dev(), generator=g)
    ws = torch.empty(gsmi.ssim_workspace_bytes(3, 80, 96), dtype=torch.uint8, device=dev())
    names = gsmi.PARAM_NAMES
    lrs = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2, "sh": 2.5e-3}
    P = _leaf_params(sc)
    mom = {k: (torch.zeros_like(P[k]), torch.zeros_like(P[k])) for k in names}
    counter = gsmi.adam_counter(dev())

    def step(rast, params, moments, count, cam_rows):
        if cam_rows is not None:
            cam_static.copy_(cam_rows)
        imgs = rast(*[params[k] for k in names])
        tg = targets.index_select(0, pick)
        loss = sum(photometric_loss(im, tg[i], 0.2, ws) for i, im in enumerate(imgs)) / 2
        loss.backward()
        gsmi.adam_step([(params[k].data, params[k].grad, moments[k][0], moments[k][1], lrs[k])
                        for k in names], sc.n, count,
                       tiles_touched=rast.frame.buffer(gsmi.BUF_TILES_TOUCHED), n_views=2)
        return loss.detach()

    # warm-up steps on a side stream, then the capture (which runs nothing)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            for t in P.values():
                t.grad = None
            step(r, P, mom, counter, table.index_select(0, pick).reshape(-1))
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for t in P.values():
        t.grad = None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        loss_static = step(r, P, mom, counter, table.index_select(0, pick).reshape(-1))
    assert int(counter[0]) == 3

    r2 = GaussianRasterizer(sc.n, cams[:2], sc.sh_degree, device=dev())
    rng = np.random.default_rng(8)
    for replay in range(4):
        pick.copy_(torch.from_numpy(rng.choice(len(cams), 2, replace=False)))
        before = {k: P[k].detach().clone() for k in names}
        mom_before = {k: (m.clone(), v.clone()) for k, (m, v) in mom.items()}
        count_before = int(counter[0])
        graph.replay()
        torch.cuda.synchronize()
        assert int(counter[0]) == count_before + 1
        assert not r.overflowed()
        # the eager step from the same state, on its own rasterizer
        P2 = {k: before[k].clone().requires_grad_() for k in names}
        mom2 = {k: (m.clone(), v.clone()) for k, (m, v) in mom_before.items()}
        r2.use_device_cameras(table.index_select(0, pick).reshape(-1))
        loss2 = step(r2, P2, mom2, count_before + 1, None)
        torch.cuda.synchronize()
        _close = lambda a, b, what: np.testing.assert_allclose(  # noqa: E731
            a.detach().cpu().double().numpy(), b.detach().cpu().double().numpy(), rtol=1e-5,
            atol=1e-5 * max(float(b.detach().abs().max()), 1e-30), err_msg="%s %d" % (what, replay))
        _close(loss_static, loss2, "loss")
        for k in names:
            _close(P[k].grad, P2[k].grad, k)
        # Adam of the replay's own gradients, counted on the host
        p3 = {k: before[k].clone() for k in names}
        m3 = {k: (m.clone(), v.clone()) for k, (m, v) in mom_before.items()}
        gsmi.adam_step([(p3[k], P[k].grad, m3[k][0], m3[k][1], lrs[k]) for k in names], sc.n,
                       count_before + 1, tiles_touched=r.frame.buffer(gsmi.BUF_TILES_TOUCHED),
                       n_views=2)
        torch.cuda.synchronize()
        for k in names:
            assert torch.equal(P[k].detach(), p3[k]), (k, replay)
            assert torch.equal(mom[k][0], m3[k][0]) and torch.equal(mom[k][1], m3[k][1]), k
        moved = sum(int((P[k].detach() != before[k]).sum()) for k in names)
        assert moved > 0, replay
