"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times: the 1,000,000-Gaussian 1600x1040 SH3 view, and the batched
coarse-to-fine frame (8 views at 400x260, 800x520 and 1600x1040, 500,000
Gaussians) with the persistent queue.

The oracle cannot render a whole full-size image in seconds, so these tests
compare what it can compute one element at a time: every projected splat,
the complete per-tile lists (they only need the projection), a random sample of
pixels, and the backward driven by a loss gradient that is non-zero only on a
random sample of pixels (then the oracle's adjoint over those pixels is the
exact reference for every splat gradient).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_20239_amd import gsmi, synth
from parity_util import (MARGIN, _check_ranges_partition, _compare_lists, assert_close_scaled,
                         check_chol, dev, gpu_forward, gpu_mean2d, raw_grad_scale, splat_view)

pytestmark = pytest.mark.gpu


def _sample_pixels(rng, W, H, m):
    flat = rng.choice(W * H, size=m, replace=False)
    return np.stack([flat % W, flat // W], 1).astype(np.int32)


@pytest.fixture(scope="module")
def view_1m_1600x1040():
    sc = synth.single_view_1m(with_targets=False)
    cam = sc.cameras[0]
    frame, flat, params, cams_dev, opts = gpu_forward(sc, [cam], opts=gsmi.raster_opts(count_composited=True),
                                                      cap=16 << 20)
    p = oracle.project(sc, cam)
    return sc, cam, frame, flat, params, cams_dev, opts, p


def test_1m_1600x1040_projection_and_tile_lists(view_1m_1600x1040):
    sc, cam, frame, flat, params, cams_dev, opts, p = view_1m_1600x1040
    nv, ni, ovf = frame.status()
    assert ovf == 0 and ni > 2_000_000
    sp = splat_view(frame)
    tt = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy().view(np.uint32)
    ok = p["flags"] == 0
    # binned: the footprint rectangle is non-empty and one of its tile squares meets
    # the footprint ellipse (a thin ellipse near the image border can have the one
    # without the other)
    vis = p["tiles_touched"] > 0
    np.testing.assert_array_equal((tt > 0)[ok], vis[ok])
    m = vis & (tt > 0)
    np.testing.assert_allclose(gpu_mean2d(sp)[m], p["mean2d"][m], rtol=1e-7, atol=1e-4)
    check_chol(sp[m, 4:7], p["conic"][m])
    np.testing.assert_allclose(sp[m, 7], p["opacity"][m], rtol=1e-6)
    np.testing.assert_allclose(sp[m, 8:11], p["rgb"][m], rtol=1e-5, atol=1e-6)
    tiles, gids, _ = oracle.tile_lists(p)
    gt = frame.buffer(gsmi.BUF_INST_TILE).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    ge = frame.buffer(gsmi.BUF_INST_ENTRY).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    gr = frame.buffer(gsmi.BUF_RANGES).cpu().numpy().view(np.uint32).reshape(-1, 2)
    _compare_lists(p, gt, ge, tiles, gids)
    _check_ranges_partition(gr, gt)


def test_1m_1600x1040_sampled_pixels(view_1m_1600x1040):
    sc, cam, frame, flat, params, cams_dev, opts, p = view_1m_1600x1040
    rng = np.random.default_rng(17)
    pix = _sample_pixels(rng, cam.width, cam.height, 2000)
    # the image corners and edges are part of every sample
    pix[:4] = [[0, 0], [cam.width - 1, 0], [0, cam.height - 1], [cam.width - 1, cam.height - 1]]
    C, T, nc, margin = oracle.render_pixels(p, pix)
    good = margin > MARGIN
    assert good.mean() > 0.98
    img = flat.view(3, cam.height, cam.width).cpu().numpy()
    got = img[:, pix[:, 1], pix[:, 0]].T
    assert_close_scaled(got[good], C[good], np.abs(C[good]), what="pixels")
    Tg = frame.buffer(gsmi.BUF_T_FINAL, torch.float32).cpu().numpy().reshape(cam.height, cam.width)
    assert_close_scaled(Tg[pix[good, 1], pix[good, 0]], T[good], np.abs(T[good]), what="T_final")
    ncg = frame.buffer(gsmi.BUF_N_COMPOSITED).cpu().numpy().view(np.uint32).reshape(cam.height,
                                                                                  cam.width)
    np.testing.assert_array_equal(ncg[pix[good, 1], pix[good, 0]], nc[good])


def test_1m_1600x1040_backward_from_sampled_pixels(view_1m_1600x1040):
    sc, cam, frame, flat, params, cams_dev, opts, p = view_1m_1600x1040
    rng = np.random.default_rng(23)
    pix = _sample_pixels(rng, cam.width, cam.height, 400)
    _, _, _, margin = oracle.render_pixels(p, pix)
    pix = pix[margin > MARGIN]
    g = rng.standard_normal((pix.shape[0], 3)).astype(np.float32)
    dL = np.zeros((3, cam.height, cam.width), np.float32)
    dL[:, pix[:, 1], pix[:, 0]] = g.T
    frame.render_backward(opts, torch.from_numpy(dL).to(dev()).reshape(-1))
    grads = gsmi.empty_grads(params)
    acc = torch.zeros(sc.n, device=dev())
    den = torch.zeros(sc.n, device=dev())
    frame.project_backward(params, sc.sh_degree, cams_dev, opts, grads, acc, den)
    torch.cuda.synchronize()
    gproj, gabs = oracle.render_backward_pixels(p, pix, g.astype(np.float64))
    sg = frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32).view(-1, 9).cpu().numpy()
    rendered = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy() > 0
    assert np.all(gabs[~rendered] == 0)
    hit = (gabs > 0).any(1)
    assert hit.sum() > 1000
    assert_close_scaled(sg[rendered], gproj[rendered], gabs[rendered], what="splat gradients")
    # the five raw-parameter gradients and the statistic against the oracle's
    # chain rule (FP64) of the oracle's splat gradients, over every Gaussian
    # whose binning is not within rounding distance of a tile decision
    racc, rden = np.zeros(sc.n), np.zeros(sc.n)
    # rendered = binned to a tile (a thin ellipse at the border can have a non-empty
    # footprint rectangle and no tile)
    rend_o = (p["tiles_touched"] > 0).astype(np.int32)
    gref = oracle.project_backward(sc, cam, rend_o, gproj, stats=(racc, rden))
    scales = raw_grad_scale(sc, cam, p, gabs)
    ok = p["flags"] == 0
    assert ok.mean() > 0.99
    for k in gsmi.PARAM_NAMES:
        g = grads[k].cpu().numpy()
        assert_close_scaled(g[..., ok], gref[k][..., ok], scales[k][..., ok], what=k)
    # the statistic counts every rendered Gaussian once
    np.testing.assert_array_equal(den.cpu().numpy(), rendered.astype(np.float32))
    np.testing.assert_array_equal(rden[ok], rendered[ok].astype(np.float64))
    gn = np.hypot(gabs[:, 0] * cam.width / 2, gabs[:, 1] * cam.height / 2)
    assert_close_scaled(acc.cpu().numpy()[ok], racc[ok], gn[ok], what="densify statistic")


@pytest.mark.parametrize("batch,persistent", [(128, 0), (64, 8192)])
def test_batched_8_views_500k_sampled(batch, persistent):
    sc = synth.batched_c2f(with_targets=False)
    cams = sc.cameras
    opts = gsmi.raster_opts(raster_batch=batch, persistent_blocks=persistent)
    frame, flat, params, cams_dev, _ = gpu_forward(sc, cams, opts=opts, cap=32 << 20)
    nv, ni, ovf = frame.status()
    assert ovf == 0
    imgs = frame.split_images(flat)
    rng = np.random.default_rng(31)
    dL = [np.zeros((3, c.height, c.width), np.float32) for c in cams]
    picks = []
    projs = []
    for v, cam in enumerate(cams):
        p = oracle.project(sc, cam)
        projs.append(p)
        pix = _sample_pixels(rng, cam.width, cam.height, 250)
        C, T, nc, margin = oracle.render_pixels(p, pix)
        good = margin > MARGIN
        got = imgs[v].view(3, cam.height, cam.width).cpu().numpy()[:, pix[:, 1], pix[:, 0]].T
        assert_close_scaled(got[good], C[good], np.abs(C[good]), what="view %d pixels" % v)
        pb = pix[good][:60]
        g = rng.standard_normal((pb.shape[0], 3)).astype(np.float32)
        dL[v][:, pb[:, 1], pb[:, 0]] = g.T
        picks.append((pb, g))
    flat_dL = torch.cat([torch.from_numpy(d).reshape(-1) for d in dL]).to(dev())
    frame.render_backward(opts, flat_dL)
    grads = gsmi.empty_grads(params)
    acc = torch.zeros(sc.n, device=dev())
    den = torch.zeros(sc.n, device=dev())
    frame.project_backward(params, sc.sh_degree, cams_dev, opts, grads, acc, den)
    torch.cuda.synchronize()
    sg = frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32).view(len(cams), sc.n, 9).cpu().numpy()
    tt = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy().reshape(len(cams), sc.n) > 0
    # the raw-parameter gradients summed over the 8 views and the statistic over
    # them, against the oracle's chain rule applied view by view
    gref, scales = None, None
    racc, rden, gn = np.zeros(sc.n), np.zeros(sc.n), np.zeros(sc.n)
    ok = np.ones(sc.n, bool)
    for v, (p, (pb, g)) in enumerate(zip(projs, picks)):
        gproj, gabs = oracle.render_backward_pixels(p, pb, g.astype(np.float64))
        assert np.all(gabs[~tt[v]] == 0)
        assert_close_scaled(sg[v][tt[v]], gproj[tt[v]], gabs[tt[v]], what="view %d grads" % v)
        gref = oracle.project_backward(sc, cams[v], (p["tiles_touched"] > 0).astype(np.int32),
                                       gproj, grads=gref, stats=(racc, rden))
        gn += np.hypot(gabs[:, 0] * cams[v].width / 2, gabs[:, 1] * cams[v].height / 2)
        sv = raw_grad_scale(sc, cams[v], p, gabs)
        scales = sv if scales is None else {k: scales[k] + sv[k] for k in sv}
        ok &= p["flags"] == 0
    assert ok.mean() > 0.99
    for k in gsmi.PARAM_NAMES:
        gk = grads[k].cpu().numpy()
        assert_close_scaled(gk[..., ok], gref[k][..., ok], scales[k][..., ok],
                            what="8-view sum " + k)
    np.testing.assert_array_equal(den.cpu().numpy(), tt.sum(0).astype(np.float32))
    np.testing.assert_array_equal(rden[ok], tt.sum(0)[ok].astype(np.float64))
    assert_close_scaled(acc.cpu().numpy()[ok], racc[ok], gn[ok], what="8-view statistic")


def test_largest_view_16384x16384():
    """The largest view the frame accepts (16384 x 16384: 1,048,576 tiles,
    268 M pixels): per-tile lists exact and sampled pixels, corners included,
    against the oracle."""
    W = H = 16384
    sc = synth.random_scene(28, 20000, W, H, sh_degree=1, log_scale=(-6.5, 0.5))
    cam = sc.cameras[0]
    frame, flat, *_ = gpu_forward(sc, [cam], cap=1 << 22)
    assert frame.T == (W // 16) * (H // 16)
    p = oracle.project(sc, cam)
    tiles, gids, _ = oracle.tile_lists(p)
    nv, ni, ovf = frame.status()
    gt = frame.buffer(gsmi.BUF_INST_TILE).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    ge = frame.buffer(gsmi.BUF_INST_ENTRY).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    _compare_lists(p, gt, ge, tiles, gids)
    assert gt.max() > (1 << 19)
    rng = np.random.default_rng(28)
    # pixels inside footprints (where the image is not background), plus random ones and the corners
    vis = np.flatnonzero(p["visible"] > 0)
    centres = np.clip(np.round(p["mean2d"][rng.choice(vis, 1500)] - 0.5), 0, W - 1).astype(np.int32)
    pix = np.concatenate([centres, _sample_pixels(rng, W, H, 496),
                          [[0, 0], [W - 1, 0], [0, H - 1], [W - 1, H - 1]]]).astype(np.int32)
    C, T, nc, margin = oracle.render_pixels(p, pix)
    good = margin > MARGIN
    assert good.mean() > 0.98 and (nc[good] > 0).sum() > 1000
    img = flat.view(3, H, W)
    got = img[:, torch.from_numpy(pix[:, 1]).long().to(img.device),
              torch.from_numpy(pix[:, 0]).long().to(img.device)].T.cpu().numpy()
    assert_close_scaled(got[good], C[good], np.abs(C[good]), what="pixels")
    Tg = frame.buffer(gsmi.BUF_T_FINAL, torch.float32).view(H, W)
    Tgot = Tg[torch.from_numpy(pix[:, 1]).long().to(Tg.device),
              torch.from_numpy(pix[:, 0]).long().to(Tg.device)].cpu().numpy()
    assert_close_scaled(Tgot[good], T[good], np.abs(T[good]), what="T_final")


def test_1m_coarse_level_200x130_both_lane_layouts():
    """The 1M-Gaussian view at 1/8 resolution, a coarse level of the
    coarse-to-fine schedule: 117 tiles whose lists hold thousands of splats,
    which the default launch renders with one pixel per lane.  Against the
    2x2-quad layout: images, final transmittance, walk lengths and composited
    counts bit-identical.  Against the oracle, in both layouts: a sample of
    pixels and the splat gradients of a loss on a sample of pixels (long
    back-to-front walks)."""
    sc = synth.single_view_1m(with_targets=False)
    cam = sc.cameras[0].scaled(8)
    p = oracle.project(sc, cam)
    rng = np.random.default_rng(31)
    pix = _sample_pixels(rng, cam.width, cam.height, 300)
    C, T, nc, margin = oracle.render_pixels(p, pix)
    good = margin > MARGIN
    assert good.mean() > 0.95
    bpix = pix[good][:150]
    g = rng.standard_normal((bpix.shape[0], 3)).astype(np.float32)
    dL = np.zeros((3, cam.height, cam.width), np.float32)
    dL[:, bpix[:, 1], bpix[:, 0]] = g.T
    gproj, gabs = oracle.render_backward_pixels(p, bpix, g.astype(np.float64))
    state = {}
    for lanes in ("pixels", "quads"):
        opts = gsmi.raster_opts(count_composited=True, lanes=lanes)
        frame, flat, *_ = gpu_forward(sc, [cam], opts=opts, cap=16 << 20)
        img = flat.view(3, cam.height, cam.width).cpu().numpy()
        got = img[:, pix[:, 1], pix[:, 0]].T
        assert_close_scaled(got[good], C[good], np.abs(C[good]), what="pixels (%s)" % lanes)
        Tg = frame.buffer(gsmi.BUF_T_FINAL, torch.float32).cpu().numpy().reshape(cam.height, cam.width)
        assert_close_scaled(Tg[pix[good, 1], pix[good, 0]], T[good], np.abs(T[good]),
                            what="T_final (%s)" % lanes)
        ncg = frame.buffer(gsmi.BUF_N_COMPOSITED).cpu().numpy().view(np.uint32)
        ncg = ncg.reshape(cam.height, cam.width)
        np.testing.assert_array_equal(ncg[pix[good, 1], pix[good, 0]], nc[good])
        frame.render_backward(opts, torch.from_numpy(dL).to(dev()).reshape(-1))
        torch.cuda.synchronize()
        sg = frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32).view(-1, 9).cpu().numpy()
        rendered = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy() > 0
        assert np.all(gabs[~rendered] == 0)
        assert (gabs > 0).any(1).sum() > 1000
        assert_close_scaled(sg[rendered], gproj[rendered], gabs[rendered],
                            what="splat gradients (%s)" % lanes)
        state[lanes] = [flat.cpu().clone(),
                        frame.buffer(gsmi.BUF_T_FINAL, torch.float32).cpu().clone(),
                        frame.buffer(gsmi.BUF_N_CONTRIB).cpu().clone(), ncg.copy()]
        del frame
    a, b = state["pixels"], state["quads"]
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)
    np.testing.assert_array_equal(a[3], b[3])
