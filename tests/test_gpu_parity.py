"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: integer / index outputs bit-exact; FP32 images and gradients within
1e-4 of the FP64 values, relative to the value or to the sum of absolute terms
that formed it (the scale FP32 summation error is proportional to).  Pixels
where a discrete decision of the compositing (alpha cutoff 1/255, clamp 0.99,
transmittance stop 1e-4) lies within 1e-5 (relative) of its threshold are
excluded from the image comparison, and their loss gradient is set to zero for
the gradient comparison, on both sides.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2507_20239_amd import gsmi, synth
from parity_util import (MARGIN, RTOL, _check_ranges_partition, _compare_lists, _norm_ranges,
                         assert_close_scaled, check_chol, dev, gpu_forward, gpu_mean2d,
                         params_of, raw_grad_scale, splat_view)

pytestmark = pytest.mark.gpu


def _scenes():
    tiny = synth.tiny_scene(seed=0, n=2000)
    rag = synth.random_scene(21, 300, 37, 29, sh_degree=3, log_scale=(-2.6, 0.5), spread=1.0)
    rag.bg = np.array([0.2, 0.4, 0.1], np.float32)
    deg1 = synth.random_scene(22, 500, 70, 45, sh_degree=1, logit=(1.5, 1.0), log_scale=(-2.2, 0.5))
    # tile lists of 676 .. 13458 instances: wave sorts in registers, LDS sorts, and LDS-sorted
    # runs merged once to three times
    dense = synth.random_scene(23, 24000, 64, 40, sh_degree=0, log_scale=(-2.6, 0.4))
    return {"tiny_2000_128x128_sh0": tiny, "ragged_300_37x29_sh3": rag, "sh1_500_70x45": deg1,
            "dense_24000_64x40_sh0": dense}


SCENES = _scenes()


@pytest.mark.parametrize("name", list(SCENES))
def test_project_matches_oracle(name):
    sc = SCENES[name]
    cam = sc.cameras[0]
    frame, *_ = gpu_forward(sc, [cam])
    p = oracle.project(sc, cam)
    tt = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy().view(np.uint32).astype(np.int64)
    key = frame.buffer(gsmi.BUF_DEPTH_KEY).cpu().numpy().view(np.uint32)
    rect = frame.buffer(gsmi.BUF_RECT).cpu().numpy().view(np.uint32).reshape(-1, 2)
    sp = splat_view(frame)
    ok = p["flags"] == 0
    assert ok.mean() > 0.99
    # binned: the footprint rectangle is non-empty and one of its tile squares meets
    # the footprint ellipse (a thin ellipse near the image border can have the one
    # without the other)
    vis = p["tiles_touched"] > 0
    # bit-exact: depth keys (all), visibility and rectangles (unflagged)
    np.testing.assert_array_equal(key[p["depth"] > 0], p["depth_key"][p["depth"] > 0])
    np.testing.assert_array_equal((tt > 0)[ok], vis[ok])
    np.testing.assert_array_equal(tt[ok], p["tiles_touched"][ok])
    r = p["rect"]
    gx0, gx1 = rect[:, 0] & 0xFFFF, rect[:, 0] >> 16
    gy0, gy1 = rect[:, 1] & 0xFFFF, rect[:, 1] >> 16
    m = ok & vis
    np.testing.assert_array_equal(np.stack([gx0, gx1, gy0, gy1], 1)[m], r[m])
    # FP32 values of visible splats
    m = vis & (tt > 0)
    np.testing.assert_allclose(gpu_mean2d(sp)[m], p["mean2d"][m], rtol=1e-7, atol=1e-5)
    check_chol(sp[m, 4:7], p["conic"][m])
    np.testing.assert_allclose(sp[m, 7], p["opacity"][m], rtol=1e-6)
    np.testing.assert_allclose(sp[m, 8:11], p["rgb"][m], rtol=1e-5, atol=1e-6)


def _border_scene(seed=31, n=20000, W=96, H=72):
    """Gaussians whose centres fall around the image border (up to 300 pixels
    outside it) and far off axis, at depths from just past the near plane,
    many of them large or elongated and some barely above the opacity cutoff:
    the cases the projection's off-screen test must leave to the exact path."""
    rng = np.random.default_rng(seed)
    base = synth.random_scene(seed, 8, W, H, sh_degree=1)
    cam = base.cameras[0]
    side = rng.integers(0, 4, n)
    d = rng.exponential(40.0, n)
    along = rng.uniform(-300, 300 + max(W, H), n)
    u = np.where(side == 0, -d, np.where(side == 1, W + d, along))
    w = np.where(side == 2, -d, np.where(side == 3, H + d, along))
    u = np.where(side >= 2, np.clip(u, -300, W + 300), u)
    w = np.where(side < 2, np.clip(w, -300, H + 300), w)
    far = rng.random(n) < 0.05   # beyond the field-of-view clamp
    u[far] *= 40.0
    z = np.where(rng.random(n) < 0.1, rng.uniform(0.21, 0.5, n), rng.uniform(0.5, 6.0, n))
    xc = (u - cam.cx) * z / cam.fx
    yc = (w - cam.cy) * z / cam.fy
    camp = np.stack([xc, yc, z])
    means = cam.R.T @ (camp - cam.t[:, None])
    log_scales = rng.uniform(-5.0, 0.0, (3, n))
    flat = rng.random(n) < 0.3
    log_scales[0, flat] -= 4.0
    logits = np.where(rng.random(n) < 0.2, rng.uniform(-5.6, -5.3, n), rng.normal(0.0, 2.0, n))
    quats = rng.standard_normal((4, n))
    sh = rng.normal(0.0, 0.3, (4, 3, n))
    f32 = lambda x: np.ascontiguousarray(x, dtype=np.float32)  # noqa: E731
    return synth.Scene(f32(means), f32(log_scales), f32(quats), f32(logits), f32(sh), 1, [cam],
                       [np.zeros((3, H, W), np.float32)], np.zeros(3, np.float32))


def test_off_screen_gaussians_project_exactly():
    """Tile counts, rectangles and depth keys of Gaussians around the image
    border against the oracle (which has no off-screen shortcut), bit for bit."""
    sc = _border_scene()
    cam = sc.cameras[0]
    frame, *_ = gpu_forward(sc, [cam])
    p = oracle.project(sc, cam)
    tt = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy().view(np.uint32).astype(np.int64)
    key = frame.buffer(gsmi.BUF_DEPTH_KEY).cpu().numpy().view(np.uint32)
    rect = frame.buffer(gsmi.BUF_RECT).cpu().numpy().view(np.uint32).reshape(-1, 2)
    ok = p["flags"] == 0
    vis = p["tiles_touched"] > 0
    # most are off screen; a good share reach into the image from outside it
    assert 0.05 < vis.mean() < 0.7 and ok.mean() > 0.99
    np.testing.assert_array_equal(key, p["depth_key"])
    np.testing.assert_array_equal(tt[ok], p["tiles_touched"][ok])
    gx0, gx1 = rect[:, 0] & 0xFFFF, rect[:, 0] >> 16
    gy0, gy1 = rect[:, 1] & 0xFFFF, rect[:, 1] >> 16
    m = ok & vis
    np.testing.assert_array_equal(np.stack([gx0, gx1, gy0, gy1], 1)[m], p["rect"][m])


@pytest.mark.parametrize("presort,balanced", [(False, False), (True, False), (False, True)])
@pytest.mark.parametrize("name", list(SCENES))
def test_binning_lists_match_oracle_exactly(name, presort, balanced):
    sc = SCENES[name]
    cam = sc.cameras[0]
    opts = gsmi.raster_opts(bg=tuple(float(x) for x in sc.bg), count_composited=True,
                            depth_presort=presort, balanced_digits=balanced)
    frame, *_ = gpu_forward(sc, [cam], opts)
    p = oracle.project(sc, cam)
    tiles, gids, ranges = oracle.tile_lists(p)
    nv, ni, ovf = frame.status()
    assert ovf == 0
    gt = frame.buffer(gsmi.BUF_INST_TILE).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    ge = frame.buffer(gsmi.BUF_INST_ENTRY).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    gr = frame.buffer(gsmi.BUF_RANGES).cpu().numpy().view(np.uint32).reshape(-1, 2)
    nflag = _compare_lists(p, gt, ge, tiles, gids)
    _check_ranges_partition(gr, gt)
    if nflag == 0:
        assert ni == tiles.size and nv == int((p["visible"] > 0).sum())
        np.testing.assert_array_equal(_norm_ranges(gr), _norm_ranges(ranges))


def test_scenes_cover_every_list_sort_path():
    # one wave with R <= 8 (<= 512) and R = 16 (<= 1024), one LDS sort (<= 2048), LDS runs merged
    # once (<= 4096), twice (<= 8192) and more
    lens = []
    for sc in SCENES.values():
        _, _, ranges = oracle.tile_lists(oracle.project(sc, sc.cameras[0]))
        lens.append(ranges[:, 1] - ranges[:, 0])
    lens = np.concatenate(lens)
    for lo, hi in ((1, 512), (512, 1024), (1024, 2048), (2048, 4096), (4096, 8192), (8192, 1 << 30)):
        assert ((lens > lo) & (lens <= hi)).any(), (lo, hi)


def _lane_opts(sc, lanes):
    return gsmi.raster_opts(bg=tuple(float(x) for x in sc.bg), count_composited=True, lanes=lanes)


# both compositing layouts: one pixel per lane (the small frames' default) and 2x2 quads
@pytest.mark.parametrize("lanes", ["pixels", "quads"])
@pytest.mark.parametrize("name", list(SCENES))
def test_render_matches_oracle(name, lanes):
    sc = SCENES[name]
    cam = sc.cameras[0]
    frame, flat, *_ = gpu_forward(sc, [cam], _lane_opts(sc, lanes))
    p = oracle.project(sc, cam)
    ref, Tref, nref, margin = oracle.render_image(p, sc.bg)
    img = flat.view(3, cam.height, cam.width).cpu().numpy()
    T = frame.buffer(gsmi.BUF_T_FINAL, torch.float32).cpu().numpy().reshape(cam.height, cam.width)
    good = margin > MARGIN
    assert good.mean() > 0.99
    scale = np.abs(ref) + np.abs(np.asarray(sc.bg, np.float64))[:, None, None]
    assert_close_scaled(img[:, good], ref[:, good], scale[:, good], what="image")
    assert_close_scaled(T[good], Tref[good], np.abs(Tref[good]), what="T_final")
    nc = frame.buffer(gsmi.BUF_N_COMPOSITED).cpu().numpy().view(np.uint32).reshape(cam.height,
                                                                                 cam.width)
    np.testing.assert_array_equal(nc[good], nref[good])


@pytest.mark.parametrize("lanes", ["pixels", "quads"])
@pytest.mark.parametrize("name", list(SCENES))
def test_backward_matches_oracle(name, lanes):
    sc = SCENES[name]
    cam = sc.cameras[0]
    frame, flat, params, cams_dev, opts = gpu_forward(sc, [cam], _lane_opts(sc, lanes))
    p = oracle.project(sc, cam)
    _, _, _, margin = oracle.render_image(p, sc.bg)
    rng = np.random.default_rng(5)
    dL = rng.standard_normal((3, cam.height, cam.width)) * 1e-3
    dL[:, margin <= MARGIN] = 0.0
    dL = dL.astype(np.float32)
    frame.render_backward(opts, torch.from_numpy(dL).to(dev()).reshape(-1))
    grads = gsmi.empty_grads(params)
    acc = torch.zeros(sc.n, device=dev())
    den = torch.zeros(sc.n, device=dev())
    frame.project_backward(params, sc.sh_degree, cams_dev, opts, grads, acc, den)
    torch.cuda.synchronize()
    gproj, gabs = oracle.render_backward_image(p, dL.astype(np.float64), sc.bg)
    sg = frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32).view(-1, 9).cpu().numpy()
    rendered = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy() > 0
    assert np.all(gabs[~rendered] == 0)
    assert_close_scaled(sg[rendered], gproj[rendered], gabs[rendered], what="splat gradients")
    racc, rden = np.zeros(sc.n), np.zeros(sc.n)
    gref = oracle.project_backward(sc, cam, p["visible"], gproj, stats=(racc, rden))
    scales = raw_grad_scale(sc, cam, p, gabs)
    for k in gsmi.PARAM_NAMES:
        assert_close_scaled(grads[k].cpu().numpy(), gref[k], scales[k], what=k)
    np.testing.assert_array_equal(den.cpu().numpy(), rden)
    gn = np.hypot(gabs[:, 0] * cam.width / 2, gabs[:, 1] * cam.height / 2)
    assert_close_scaled(acc.cpu().numpy(), racc, gn, what="densify statistic")


def test_multiview_frame_matches_per_view_oracle():
    sc = synth.random_scene(23, 400, 48, 40, sh_degree=2, n_views=3, log_scale=(-2.5, 0.5))
    cams = [sc.cameras[0], sc.cameras[1].scaled(2), sc.cameras[2]]
    cams[2] = synth.Camera(cams[2].R, cams[2].t, cams[2].fx, cams[2].fy, 20.5, 17.0, 41, 35)
    frame, flat, params, cams_dev, opts = gpu_forward(sc, cams)
    imgs = frame.split_images(flat)
    ranges = frame.buffer(gsmi.BUF_RANGES).cpu().numpy().view(np.uint32).reshape(-1, 2)
    nv, ni, _ = frame.status()
    gt = frame.buffer(gsmi.BUF_INST_TILE).cpu().numpy()[:ni].view(np.uint32)
    ge = frame.buffer(gsmi.BUF_INST_ENTRY).cpu().numpy()[:ni].view(np.uint32)
    base = 0
    for v, cam in enumerate(cams):
        p = oracle.project(sc, cam)
        ref, _, _, margin = oracle.render_image(p)
        good = margin > MARGIN
        got = imgs[v].cpu().numpy()
        assert_close_scaled(got[:, good], ref[:, good], np.abs(ref[:, good]), what="view %d" % v)
        tiles, gids, rr = oracle.tile_lists(p, tile_base=base)
        T = rr.shape[0]
        sel = (gt >= base) & (gt < base + T)
        _compare_lists(p, gt[sel].astype(np.int64), ge[sel].astype(np.int64), tiles, gids,
                       entry_base=v * sc.n)
        base += T
    _check_ranges_partition(ranges, gt.astype(np.int64))
    assert base == frame.T


def test_thirty_two_views_in_one_frame():
    """The largest frame (32 views, mixed sizes): every view's image and tile
    lists against the oracle, and the adjoint summed over the views with the
    statistic counting each view that renders a Gaussian."""
    sc = synth.random_scene(26, 300, 40, 30, sh_degree=1, n_views=32, log_scale=(-2.3, 0.5))
    cams = [c.scaled(2) if v % 3 == 1 else c for v, c in enumerate(sc.cameras)]
    assert len(cams) == gsmi.MAX_VIEWS
    frame, flat, params, cams_dev, opts = gpu_forward(sc, cams)
    imgs = frame.split_images(flat)
    nv, ni, _ = frame.status()
    gt = frame.buffer(gsmi.BUF_INST_TILE).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    ge = frame.buffer(gsmi.BUF_INST_ENTRY).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    rng = np.random.default_rng(26)
    dLs, projs, base = [], [], 0
    for v, cam in enumerate(cams):
        p = oracle.project(sc, cam)
        ref, _, _, margin = oracle.render_image(p)
        good = margin > MARGIN
        got = imgs[v].cpu().numpy()
        assert_close_scaled(got[:, good], ref[:, good], np.abs(ref[:, good]), what="view %d" % v)
        tiles, gids, rr = oracle.tile_lists(p, tile_base=base)
        sel = (gt >= base) & (gt < base + rr.shape[0])
        _compare_lists(p, gt[sel], ge[sel], tiles, gids, entry_base=v * sc.n)
        base += rr.shape[0]
        dL = rng.standard_normal((3, cam.height, cam.width)) * 1e-3
        dL[:, ~good] = 0.0
        dLs.append(dL.astype(np.float32))
        projs.append(p)
    assert base == frame.T
    frame.render_backward(opts, torch.from_numpy(np.concatenate([d.reshape(-1) for d in dLs])).to(dev()))
    grads = gsmi.empty_grads(params)
    acc = torch.zeros(sc.n, device=dev())
    den = torch.zeros(sc.n, device=dev())
    frame.project_backward(params, sc.sh_degree, cams_dev, opts, grads, acc, den)
    torch.cuda.synchronize()
    want = {k: 0.0 for k in gsmi.PARAM_NAMES}
    scale = {k: 0.0 for k in gsmi.PARAM_NAMES}
    racc, rden = np.zeros(sc.n), np.zeros(sc.n)
    for cam, p, dL in zip(cams, projs, dLs):
        gproj, gabs = oracle.render_backward_image(p, dL.astype(np.float64))
        g = oracle.project_backward(sc, cam, p["visible"], gproj, stats=(racc, rden))
        s = raw_grad_scale(sc, cam, p, gabs)
        for k in gsmi.PARAM_NAMES:
            want[k] = want[k] + g[k]
            scale[k] = scale[k] + s[k]
    for k in gsmi.PARAM_NAMES:
        assert_close_scaled(grads[k].cpu().numpy(), want[k], scale[k], what=k)
    np.testing.assert_array_equal(den.cpu().numpy(), rden)


def test_empty_and_culled_scene_renders_background():
    sc = synth.random_scene(24, 64, 33, 17, sh_degree=0)
    sc.means[2] = -1.0          # every Gaussian behind the camera
    sc.bg = np.array([0.3, 0.6, 0.9], np.float32)
    frame, flat, params, cams_dev, opts = gpu_forward(sc, sc.cameras)
    nv, ni, ovf = frame.status()
    assert nv == 0 and ni == 0 and ovf == 0
    img = flat.view(3, 17, 33).cpu().numpy()
    for c in range(3):
        assert np.all(img[c] == sc.bg[c])
    dL = torch.ones(flat.numel(), device=dev())
    frame.render_backward(opts, dL)
    grads = gsmi.empty_grads(params)
    frame.project_backward(params, 0, cams_dev, opts, grads)
    for k in gsmi.PARAM_NAMES:
        assert torch.count_nonzero(grads[k]).item() == 0
    # the fused forms: the L1 term of the background alone, and an optimiser
    # step that moves nothing (no Gaussian was rendered)
    loss = torch.zeros(1, device=dev())
    img2, g2 = torch.empty_like(flat), torch.empty_like(flat)
    frame.composite_l1(opts, img2, torch.zeros_like(flat), 0.5, loss, g2)
    torch.cuda.synchronize()
    assert torch.equal(img2, flat) and bool((g2 == 0.5).all())
    assert float(loss) == pytest.approx(0.5 * 17 * 33 * float(sc.bg.sum()), rel=1e-6)
    before = {k: t.clone() for k, t in params.items()}
    mom = {k: (torch.full_like(t, 0.1), torch.full_like(t, 0.2)) for k, t in params.items()}
    lrs = {k: 1e-3 for k in gsmi.PARAM_NAMES}
    frame.project_backward(params, 0, cams_dev, opts, {}, adam=gsmi.FusedAdamStep(mom, lrs, 1))
    torch.cuda.synchronize()
    for k in gsmi.PARAM_NAMES:
        assert torch.equal(params[k], before[k]), k
        assert bool((mom[k][0] == 0.1).all()) and bool((mom[k][1] == 0.2).all()), k


def test_nonfinite_gaussians_are_culled():
    """Gaussians with a NaN mean, log-scale or opacity, an infinite mean, or a
    zero quaternion get no tiles, and the image equals that of the scene
    without them, bit for bit (the others keep their relative order)."""
    sc = synth.random_scene(25, 600, 70, 45, sh_degree=1, log_scale=(-2.2, 0.5))
    rng = np.random.default_rng(25)
    bad = rng.choice(sc.n, 50, replace=False)
    sc.means[0, bad[:10]] = np.nan
    sc.means[2, bad[10:20]] = np.inf
    sc.log_scales[1, bad[20:30]] = np.nan
    sc.quats[:, bad[30:40]] = 0.0
    sc.opacity_logits[bad[40:]] = np.nan
    keep = np.setdiff1d(np.arange(sc.n), bad)
    clean = synth.Scene(sc.means[:, keep].copy(), sc.log_scales[:, keep].copy(),
                        sc.quats[:, keep].copy(), sc.opacity_logits[keep].copy(),
                        sc.sh[:, :, keep].copy(), sc.sh_degree, sc.cameras, [], sc.bg)
    cam = sc.cameras[0]
    frame, img, *_ = gpu_forward(sc, [cam])
    tt = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy()[: sc.n]
    assert not tt[bad].any() and tt[keep].any()
    _, img_clean, *_ = gpu_forward(clean, [cam])
    assert torch.isfinite(img).all()
    assert torch.equal(img, img_clean)


def test_capacity_overflow_is_reported_and_bounded():
    sc = SCENES["tiny_2000_128x128_sh0"]
    cam = sc.cameras[0]
    frame, flat, *_ = gpu_forward(sc, [cam], cap=1000)
    nv, ni, ovf = frame.status(raise_on_overflow=False)
    assert ovf == 1 and ni > 1000
    with pytest.raises(gsmi.GsError):
        frame.status()


@pytest.mark.parametrize("n,wraps", [((1 << 20) - 1, False), ((1 << 20) + 1, True)])
def test_instance_totals_at_and_beyond_2_to_32(n, wraps):
    """n Gaussians that each cover all 4096 tiles of a 1024x1024 view: 2^32 - 4096
    instances is an ordinary overflow with the exact total; 2^32 + 4096 (whose
    low 32 bits would look like a small total) is reported as an overflow with
    nothing kept, and the view renders as background."""
    rng = np.random.default_rng(27)
    means = np.stack([rng.uniform(-1e-3, 1e-3, n), rng.uniform(-1e-3, 1e-3, n),
                      np.full(n, 3.0)]).astype(np.float32)
    sc = synth.Scene(means, np.full((3, n), 1.5, np.float32), np.tile([[1.0], [0], [0], [0]], n).astype(np.float32),
                     np.zeros(n, np.float32), np.full((1, 3, n), 0.3, np.float32), 0,
                     [synth.Camera(np.eye(3), np.zeros(3), 1024.0, 1024.0, 512.0, 512.0, 1024, 1024)],
                     [], np.array([0.25, 0.5, 0.75], np.float32))
    frame, flat, *_ = gpu_forward(sc, sc.cameras, cap=1 << 20)
    tt = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy().view(np.uint32)
    assert (tt == 4096).all()
    nv, ni, ovf = frame.status(raise_on_overflow=False)
    assert ovf == 1
    with pytest.raises(gsmi.GsError):
        frame.status()
    if wraps:
        assert ni == 0xFFFFFFFF and nv <= n
        img = flat.view(3, 1024, 1024).cpu().numpy()
        for c in range(3):
            assert np.all(img[c] == sc.bg[c])
    else:
        assert ni == 4096 * n and nv == n


def test_counting_composited_splats_changes_nothing_else():
    sc = SCENES["ragged_300_37x29_sh3"]
    cam = sc.cameras[0]
    bufs = (gsmi.BUF_T_FINAL, gsmi.BUF_N_CONTRIB)
    out = []
    for count in (False, True):
        o = gsmi.raster_opts(bg=tuple(sc.bg), count_composited=count)
        frame, img, *_ = gpu_forward(sc, [cam], o)
        out.append([img.clone()] + [frame.buffer(b).clone() for b in bufs])
    for a, b in zip(*out):
        assert torch.equal(a, b)


def test_persistent_queue_gives_identical_images():
    sc = SCENES["ragged_300_37x29_sh3"]
    cam = sc.cameras[0]
    o1 = gsmi.raster_opts(bg=tuple(sc.bg))
    o2 = gsmi.raster_opts(bg=tuple(sc.bg), persistent_blocks=7, raster_batch=64)
    _, a, *_ = gpu_forward(sc, [cam], o1)
    _, b, *_ = gpu_forward(sc, [cam], o2)
    assert torch.equal(a, b)


@pytest.mark.parametrize("n,bits", [(0, 32), (1, 32), (100, 7), (4097, 16), (70001, 32),
                                    (1_000_003, 24)])
def test_radix_sort_is_stable_and_exact(n, bits):
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 2 ** bits, n, dtype=np.uint64).astype(np.uint32)
    if n > 10:
        keys[: n // 3] = keys[n // 2]     # many ties
    vals = np.arange(n, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int32).copy()).to(dev())
    vt = torch.from_numpy(vals.view(np.int32).copy()).to(dev())
    gsmi.sort_pairs(kt, vt, bits)
    order = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(kt.cpu().numpy().view(np.uint32), keys[order])
    np.testing.assert_array_equal(vt.cpu().numpy().view(np.uint32), vals[order])


def test_l1_loss_grad():
    rng = np.random.default_rng(3)
    a = rng.random(100_003).astype(np.float32)
    b = rng.random(100_003).astype(np.float32)
    b[:10] = a[:10]
    loss, g = gsmi.l1_loss_grad(torch.from_numpy(a).to(dev()), torch.from_numpy(b).to(dev()),
                                1.0 / a.size)
    ref_loss, ref_g = oracle.l1_loss_grad(a, b)
    assert float(loss.item()) == pytest.approx(ref_loss, rel=1e-5)
    np.testing.assert_array_equal(g.cpu().numpy(), ref_g.astype(np.float32))


@pytest.mark.parametrize("lanes,persistent", [("pixels", 0), ("quads", 0), (None, 7)])
def test_composite_l1_equals_composite_then_l1(lanes, persistent):
    """gs_composite_l1 (the L1 term of Eq. 3 computed as the compositing writes
    each pixel) against gs_composite followed by gs_l1_loss_grad on a two-view
    frame with ragged edges and pixels equal to their target: images, final
    transmittance, walk lengths and dL/dimage bit for bit, the loss to FP32
    summation order; the loss is added to what the caller set."""
    sc = synth.random_scene(27, 3000, 150, 100, sh_degree=2, n_views=2, log_scale=(-2.5, 0.5))
    cams = [sc.cameras[0], synth.Camera(sc.cameras[1].R, sc.cameras[1].t, 90.0, 90.0, 45.3,
                                        30.8, 91, 61)]
    opts = gsmi.raster_opts(bg=(0.1, 0.2, 0.3), lanes=lanes, persistent_blocks=persistent)
    frame, flat, *_ = gpu_forward(sc, cams, opts)
    torch.cuda.synchronize()
    ref_img = flat.clone()
    ref_T = frame.buffer(gsmi.BUF_T_FINAL, torch.float32).clone()
    ref_n = frame.buffer(gsmi.BUF_N_CONTRIB).clone()
    g = torch.Generator(device=dev())
    g.manual_seed(13)
    targets = torch.rand(flat.numel(), device=dev(), generator=g)
    targets[::97] = ref_img[::97]   # sign(0) = 0
    scale = 1.0 / flat.numel()
    ref_loss, ref_dL = gsmi.l1_loss_grad(ref_img, targets, scale)
    img = torch.empty_like(flat)
    dL = torch.empty_like(flat)
    loss = torch.full((1,), 0.25, device=dev())
    frame.composite_l1(opts, img, targets, scale, loss, dL)
    torch.cuda.synchronize()
    assert torch.equal(img, ref_img)
    assert torch.equal(frame.buffer(gsmi.BUF_T_FINAL, torch.float32), ref_T)
    assert torch.equal(frame.buffer(gsmi.BUF_N_CONTRIB), ref_n)
    assert torch.equal(dL, ref_dL)
    assert int((dL == 0).sum()) >= flat.numel() // 97
    assert float(loss) - 0.25 == pytest.approx(float(ref_loss), rel=1e-5)


def test_render_twice_after_one_projection_is_identical():
    """Rendering reads the projection's outputs without modifying them, so a
    second render of the same projection repeats the first exactly."""
    sc = SCENES["sh1_500_70x45"]
    cam = sc.cameras[0]
    frame, a, params, cams_dev, opts = gpu_forward(sc, [cam])
    a = a.clone()
    b = frame.render(opts)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_persistent_backward_after_plain_render_is_rejected_on_the_host():
    """A persistent adjoint walks the heavy-first tile order, which only a
    persistent render builds.  After a plain render the call is refused by
    host-side validation (nothing is launched), and the frame stays usable."""
    sc = SCENES["sh1_500_70x45"]
    cam = sc.cameras[0]
    plain = gsmi.raster_opts(bg=tuple(sc.bg))
    pers = gsmi.raster_opts(bg=tuple(sc.bg), persistent_blocks=16)
    frame, img, params, cams_dev, _ = gpu_forward(sc, [cam], plain)
    dL = torch.full_like(img, 1e-3)
    L = gsmi.lib()
    st = L.gs_render_backward(frame.handle, ctypes.byref(pers), gsmi._ptr(dL), gsmi._stream())
    assert st == gsmi.GS_ERR_INVALID
    assert b"heavy-first" in L.gs_last_error()
    # the same frame then runs both adjoints once the persistent render built the order
    frame.render_backward(plain, dL)
    a = frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32).clone()
    frame.project(params, sc.sh_degree, cams_dev, pers)
    frame.render(pers, img)
    frame.render_backward(pers, dL)
    torch.cuda.synchronize()
    b = frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32)
    tt = frame.buffer(gsmi.BUF_TILES_TOUCHED).view(-1) > 0
    ga, gb = a.view(-1, 9)[tt], b.view(-1, 9)[tt]
    assert torch.allclose(ga, gb, rtol=1e-4, atol=1e-6 * float(ga.abs().max()))


def _quadrant_edge_scene(seed=41, n=6000, W=160, H=112):
    """Small and elongated Gaussians centred on and next to the 8-pixel
    quadrant lines and the 16-pixel tile lines, with opacities from just above
    the 1/255 cutoff to 1: the splats whose quadrant masks decide the most
    (pixel lanes walk only the splats meeting their quadrant)."""
    rng = np.random.default_rng(seed)
    base = synth.random_scene(seed, 8, W, H, sh_degree=1)
    cam = base.cameras[0]
    u = 8.0 * rng.integers(0, W // 8 + 1, n) + rng.choice([0.0, 0.5, -0.5, 1e-3, -1e-3, 2.0], n)
    w = 8.0 * rng.integers(0, H // 8 + 1, n) + rng.choice([0.0, 0.5, -0.5, 1e-3, -1e-3, 2.0], n)
    z = rng.uniform(1.0, 4.0, n)
    camp = np.stack([(u - cam.cx) * z / cam.fx, (w - cam.cy) * z / cam.fy, z])
    means = cam.R.T @ (camp - cam.t[:, None])
    log_scales = rng.uniform(-5.5, -2.5, (3, n))
    thin = rng.random(n) < 0.4
    log_scales[0, thin] -= 3.0
    logits = np.where(rng.random(n) < 0.3, rng.uniform(-5.6, -5.0, n), rng.normal(0.0, 2.0, n))
    f32 = lambda x: np.ascontiguousarray(x, dtype=np.float32)  # noqa: E731
    return synth.Scene(f32(means), f32(log_scales), f32(rng.standard_normal((4, n))), f32(logits),
                       f32(rng.normal(0.0, 0.3, (4, 3, n))), 1, [cam],
                       [np.zeros((3, H, W), np.float32)], np.zeros(3, np.float32))


def _tall_scene(seed=43, n_small=3000, n_tall=40, W=512, H=8192):
    """A tall view (32 x 512 tiles) with small Gaussians and a few long
    axis-aligned ones whose footprints span up to all 512 tile rows, so the
    emission's row counting needs several passes for one chunk of instances
    and starts chunks in the middle of a footprint."""
    rng = np.random.default_rng(seed)
    cam = synth.random_scene(seed, 8, W, H, sh_degree=1).cameras[0]
    n = n_small + n_tall
    u = rng.uniform(-20.0, W + 20.0, n)
    w = rng.uniform(-20.0, H + 20.0, n)
    z = rng.uniform(1.5, 4.0, n)
    camp = np.stack([(u - cam.cx) * z / cam.fx, (w - cam.cy) * z / cam.fy, z])
    means = cam.R.T @ (camp - cam.t[:, None])
    log_scales = rng.uniform(-4.0, -1.5, (3, n))
    quats = rng.standard_normal((4, n))
    t = slice(n_small, n)
    log_scales[0, t] = rng.uniform(-3.0, -1.5, n_tall)
    log_scales[1, t] = rng.uniform(0.5, 2.0, n_tall)
    log_scales[2, t] = -3.0
    quats[:, t] = np.array([1.0, 0.0, 0.0, 0.0])[:, None]
    logits = rng.normal(1.0, 1.5, n)
    f32 = lambda x: np.ascontiguousarray(x, dtype=np.float32)  # noqa: E731
    return synth.Scene(f32(means), f32(log_scales), f32(quats), f32(logits),
                       f32(rng.normal(0.0, 0.3, (4, 3, n))), 1, [cam],
                       [np.zeros((3, H, W), np.float32)], np.zeros(3, np.float32))


@pytest.mark.parametrize("presort", [False, True])
def test_emission_of_footprints_spanning_hundreds_of_rows(presort):
    """Footprints of up to 512 tile rows, next to small ones: the per-tile
    lists bit-exact against the oracle whichever way the emission places a
    chunk's instances (row counts in several passes for chunks of few large
    footprints, each instance walking its footprint's rows for chunks of many
    small ones), in entry and in depth order."""
    sc = _tall_scene()
    cam = sc.cameras[0]
    p = oracle.project(sc, cam)
    rect = p["rect"][p["tiles_touched"] > 0]
    assert (rect[:, 3] - rect[:, 2] + 1).max() > 256   # one footprint outgrows a pass
    opts = gsmi.raster_opts(count_composited=True, depth_presort=presort)
    frame, *_ = gpu_forward(sc, [cam], opts, cap=1 << 20)
    tiles, gids, ranges = oracle.tile_lists(p)
    nv, ni, ovf = frame.status()
    assert ovf == 0
    gt = frame.buffer(gsmi.BUF_INST_TILE).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    ge = frame.buffer(gsmi.BUF_INST_ENTRY).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    gr = frame.buffer(gsmi.BUF_RANGES).cpu().numpy().view(np.uint32).reshape(-1, 2)
    nflag = _compare_lists(p, gt, ge, tiles, gids)
    _check_ranges_partition(gr, gt)
    if nflag == 0:
        assert ni == tiles.size
        np.testing.assert_array_equal(_norm_ranges(gr), _norm_ranges(ranges))


@pytest.mark.parametrize("sigma3", [False, True])
def test_quadrant_walk_is_exact(sigma3):
    """Pixel lanes walk only the splats whose footprint meets their 8x8
    quadrant; quads walk every splat of the list.  On splats sitting on the
    quadrant and tile lines both give bit-identical images, transmittance,
    walk lengths and composited counts (a splat skipped wrongly would change
    them), and the same gradients up to FP32 summation order; under the
    3-sigma footprint the lists hold splats the ellipse test excludes."""
    sc = _quadrant_edge_scene()
    cams = sc.cameras
    out = {}
    dL = None
    for lanes in ("pixels", "quads"):
        opts = gsmi.raster_opts(bg=(0.1, 0.2, 0.3), count_composited=True, lanes=lanes,
                                footprint_3sigma=sigma3)
        frame, flat, *_ = gpu_forward(sc, cams, opts)
        if dL is None:
            rng = np.random.default_rng(3)
            dL = torch.from_numpy(rng.standard_normal(flat.numel()).astype(np.float32)).to(dev())
        frame.render_backward(opts, dL)
        torch.cuda.synchronize()
        out[lanes] = dict(img=flat.clone(),
                          T=frame.buffer(gsmi.BUF_T_FINAL, torch.float32).clone(),
                          n=frame.buffer(gsmi.BUF_N_CONTRIB).clone(),
                          nc=frame.buffer(gsmi.BUF_N_COMPOSITED).clone(),
                          g=frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32).view(-1, 9).clone(),
                          tt=frame.buffer(gsmi.BUF_TILES_TOUCHED).clone())
    a, b = out["pixels"], out["quads"]
    assert int((a["nc"] > 0).sum()) > 1000
    for k in ("img", "T", "n", "nc", "tt"):
        assert torch.equal(a[k], b[k]), k
    r = a["tt"] > 0
    ga, gb = a["g"][r].double(), b["g"][r].double()
    scale = gb.abs().max(dim=0).values.clamp_min(1e-30)
    assert ((ga - gb).abs() <= 1e-5 * scale + 1e-5 * gb.abs()).all()


def test_lane_layouts_agree():
    """One pixel per lane and 2x2 quads per lane: images, final transmittance,
    walk lengths and composited counts bit-identical (each pixel's arithmetic
    is the same) and equal to the default layout's, splat gradients equal to
    FP32 summation order, on a two-view frame with ragged edges.  Host validation refuses both layouts at once and
    one pixel per lane on a persistent grid."""
    sc = synth.random_scene(27, 3000, 150, 100, sh_degree=2, n_views=2, log_scale=(-2.5, 0.5))
    cams = [sc.cameras[0], synth.Camera(sc.cameras[1].R, sc.cameras[1].t, 90.0, 90.0, 45.3,
                                        30.8, 91, 61)]
    out = {}
    rng = np.random.default_rng(9)
    dL = None
    for lanes in ("pixels", "quads", None):
        opts = _lane_opts(sc, lanes)
        frame, flat, *_ = gpu_forward(sc, cams, opts)
        if dL is None:
            dL = torch.from_numpy(rng.standard_normal(flat.numel()).astype(np.float32) * 1e-3)
            dL = dL.to(dev())
        frame.render_backward(opts, dL)
        torch.cuda.synchronize()
        out[lanes] = dict(img=flat.clone(),
                          T=frame.buffer(gsmi.BUF_T_FINAL, torch.float32).clone(),
                          n=frame.buffer(gsmi.BUF_N_CONTRIB).clone(),
                          nc=frame.buffer(gsmi.BUF_N_COMPOSITED).clone(),
                          g=frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32).view(-1, 9).clone(),
                          tt=frame.buffer(gsmi.BUF_TILES_TOUCHED).clone())
    a, b, c = out["pixels"], out["quads"], out[None]
    for k in ("img", "T", "n", "nc", "tt"):
        assert torch.equal(a[k], b[k]), k
        assert torch.equal(a[k], c[k]), k
    r = a["tt"] > 0
    ga, gb = a["g"][r].double(), b["g"][r].double()
    scale = gb.abs().max(dim=0).values.clamp_min(1e-30)
    assert ((ga - gb).abs() <= 1e-5 * scale + 1e-5 * gb.abs()).all()
    gc = c["g"][r].double()
    assert ((gc - ga).abs() <= 1e-5 * scale + 1e-5 * ga.abs()).all()
    L = gsmi.lib()
    frame, flat, *_ = gpu_forward(sc, cams, _lane_opts(sc, None))
    for flags, pb in ((gsmi.RASTER_LANE_PIXELS | gsmi.RASTER_LANE_QUADS, 0),
                      (gsmi.RASTER_LANE_PIXELS, 16)):
        o = _lane_opts(sc, None)
        o.flags |= flags
        o.persistent_blocks = pb
        st = L.gs_composite(frame.handle, ctypes.byref(o), gsmi._ptr(flat), gsmi._stream())
        assert st == gsmi.GS_ERR_INVALID, flags
        assert b"pixel" in L.gs_last_error().lower() or b"lane" in L.gs_last_error().lower()


def test_bin_then_composite_is_render():
    """gs_bin followed by gs_composite gives gs_render's image and per-pixel
    state bit for bit (plain and persistent); a persistent composite after a
    plain binning is refused on the host."""
    sc = SCENES["ragged_300_37x29_sh3"]
    cam = sc.cameras[0]
    for pb in (0, 5):
        o = gsmi.raster_opts(bg=tuple(sc.bg), persistent_blocks=pb, count_composited=True)
        frame, a, params, cams_dev, _ = gpu_forward(sc, [cam], o)
        bufs = [frame.buffer(b).clone() for b in (gsmi.BUF_T_FINAL, gsmi.BUF_N_CONTRIB,
                                                  gsmi.BUF_N_COMPOSITED)]
        a = a.clone()
        frame.project(params, sc.sh_degree, cams_dev, o)
        frame.bin(o)
        b = frame.composite(o)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        for x, b2 in zip(bufs, (gsmi.BUF_T_FINAL, gsmi.BUF_N_CONTRIB, gsmi.BUF_N_COMPOSITED)):
            assert torch.equal(x, frame.buffer(b2))
    plain = gsmi.raster_opts(bg=tuple(sc.bg))
    frame.bin(plain)
    with pytest.raises(gsmi.GsError, match="heavy-first"):
        frame.composite(gsmi.raster_opts(bg=tuple(sc.bg), persistent_blocks=5))


def test_sticky_overflow_flag():
    """The sticky flag records an overflowing binning until the caller clears
    it, while the per-render flag follows the last binning."""
    sc = SCENES["sh1_500_70x45"]
    cam = sc.cameras[0]
    o = gsmi.raster_opts(bg=tuple(sc.bg))
    frame, _, params, cams_dev, _ = gpu_forward(sc, [cam], o, cap=1 << 20)
    assert not frame.overflowed()
    small = gsmi.Frame(sc.n, [(cam.width, cam.height)], 64, dev())
    small.project(params, sc.sh_degree, cams_dev, o)
    small.render(o)
    assert small.status(raise_on_overflow=False)[2] == 1
    assert small.overflowed()
    assert small.overflowed(clear=True) and not small.overflowed()
    # the flag stays clear across renders that fit
    empty = synth.random_scene(3, 4, cam.width, cam.height, sh_degree=1)
    small2 = gsmi.Frame(empty.n, [(cam.width, cam.height)], 64, dev())
    small2.project(params_of(empty), empty.sh_degree, cams_dev, o)
    small2.render(o)
    assert not small2.overflowed()


@pytest.mark.parametrize("name", ["sh1_500_70x45", "long_lists_3000_96x64"])
def test_depth_presort_gives_the_same_lists_images_and_gradients(name):
    """Ordering the visible entries by depth before emission (the presort
    path) leaves the per-tile lists, images, per-pixel state and splat
    gradients bit-identical to sorting each tile's list afterwards."""
    sc = SCENES[name] if name in SCENES else synth.random_scene(9, 3000, 96, 64, sh_degree=1,
                                                                 log_scale=(-1.8, 0.4))
    cam = sc.cameras[0]
    out = []
    for presort in (False, True):
        o = gsmi.raster_opts(bg=tuple(sc.bg), count_composited=True, depth_presort=presort)
        frame, img, *_ = gpu_forward(sc, [cam], o)
        nv, ni, ovf = frame.status()
        dL = torch.linspace(-1e-3, 1e-3, img.numel(), device=img.device)
        frame.render_backward(o, dL)
        torch.cuda.synchronize()
        bufs = [frame.buffer(b).clone() for b in (gsmi.BUF_RANGES, gsmi.BUF_T_FINAL,
                                                  gsmi.BUF_N_CONTRIB, gsmi.BUF_N_COMPOSITED)]
        lists = [frame.buffer(b)[:ni].clone() for b in (gsmi.BUF_INST_TILE, gsmi.BUF_INST_ENTRY)]
        out.append([img.clone()] + bufs + lists +
                   [frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32).clone()])
    for a, b in zip(out[0][:-1], out[1][:-1]):
        assert torch.equal(a, b)
    # the splat gradients are sums of hardware atomics (order not fixed)
    ga, gb = out[0][-1], out[1][-1]
    assert torch.allclose(ga, gb, rtol=1e-5, atol=1e-6 * float(ga.abs().max()))


def test_gradients_of_rendered_rows_only():
    """With GS_RASTER_GRAD_RENDERED_ONLY the projection adjoint writes the rows
    of rendered Gaussians (bit-identical to the dense call's rows) and leaves
    the others as they were; waves with no rendered Gaussian are skipped."""
    sc = synth.random_scene(43, 6000, 96, 64, sh_degree=3, spread=2.5)
    cam = sc.cameras[0]
    params = params_of(sc)
    src, kind = gsmi.spatial_order(params["means"])
    params = dict(zip(gsmi.PARAM_NAMES, gsmi.reorder([params[k] for k in gsmi.PARAM_NAMES], src,
                                                     kind)))
    cams = gsmi.cameras_to_device([cam], dev())
    dense = gsmi.raster_opts(bg=tuple(sc.bg))
    sparse = gsmi.raster_opts(bg=tuple(sc.bg), grad_rendered_only=True)
    frame = gsmi.Frame(sc.n, [(cam.width, cam.height)], 1 << 22, dev())
    frame.project(params, sc.sh_degree, cams, dense)
    img = frame.render(dense)
    frame.render_backward(dense, torch.linspace(-1e-3, 1e-3, img.numel(), device=dev()))
    out = []
    for o in (dense, sparse):
        grads = {k: torch.full_like(v, 7.0) for k, v in params.items()}
        frame.project_backward(params, sc.sh_degree, cams, o, grads)
        torch.cuda.synchronize()
        out.append(grads)
    rend = frame.buffer(gsmi.BUF_TILES_TOUCHED).view(-1) > 0
    # waves (64 consecutive Gaussians) with a rendered one are written whole
    pad = torch.zeros((sc.n + 63) // 64 * 64, dtype=torch.bool, device=dev())
    pad[: sc.n] = rend
    written = pad.view(-1, 64).any(1).repeat_interleave(64)[: sc.n]
    assert (~written).any() and written.any()
    for k in gsmi.PARAM_NAMES:
        d, s = out[0][k], out[1][k]
        assert torch.equal(d[..., written], s[..., written]), k
        assert bool((s[..., ~written] == 7.0).all()), k
        assert bool((d[..., ~rend] == 0).all()), k
