"""The 3-sigma footprint (GS_RASTER_FOOTPRINT_3SIGMA: the original 3DGS binning,
every Gaussian in front of the camera binned to the tiles its 3-sigma square
meets) against the oracle's: rectangles, tile counts and per-tile lists
bit-exact, images, transmittance and composited counts, and the gradients
within the FP32 bounds of the default footprint's suite."""
import numpy as np
import pytest
import torch

import oracle
from paper_2507_20239_amd import gsmi, synth
from parity_util import (MARGIN, _check_ranges_partition, _compare_lists, _norm_ranges,
                         assert_close_scaled, dev, gpu_forward, raw_grad_scale)

pytestmark = pytest.mark.gpu


def _scenes():
    # opaque splats of several pixels (the 1/255 ellipse outgrows the square), and a
    # mix with many splats below 1/255 (binned here, never composited)
    large = synth.random_scene(31, 300, 70, 45, sh_degree=1, logit=(3.0, 1.0), log_scale=(-1.2, 0.4))
    large.bg = np.array([0.2, 0.4, 0.1], np.float32)
    faint = synth.random_scene(32, 2000, 96, 64, sh_degree=2, logit=(-2.0, 3.0),
                               log_scale=(-2.4, 0.6))
    return {"large_300_70x45_sh1": large, "faint_2000_96x64_sh2": faint}


SCENES = _scenes()


def _opts(sc, footprint_3sigma=True):
    return gsmi.raster_opts(bg=tuple(float(x) for x in sc.bg), count_composited=True,
                            footprint_3sigma=footprint_3sigma)


@pytest.mark.parametrize("name", list(SCENES))
def test_3sigma_rectangles_and_lists_match_oracle(name):
    sc = SCENES[name]
    cam = sc.cameras[0]
    frame, *_ = gpu_forward(sc, [cam], _opts(sc))
    p = oracle.project(sc, cam, footprint="3sigma")
    ok = p["flags"] == 0
    assert ok.mean() > 0.99
    tt = frame.buffer(gsmi.BUF_TILES_TOUCHED).cpu().numpy().view(np.uint32).astype(np.int64)
    rect = frame.buffer(gsmi.BUF_RECT).cpu().numpy().view(np.uint32).reshape(-1, 2)
    np.testing.assert_array_equal(tt[ok], p["tiles_touched"][ok])
    m = ok & (p["visible"] > 0)
    got = np.stack([rect[:, 0] & 0xFFFF, rect[:, 0] >> 16, rect[:, 1] & 0xFFFF, rect[:, 1] >> 16], 1)
    np.testing.assert_array_equal(got[m], p["rect"][m])
    if name.startswith("faint"):
        assert (p["opacity"][p["visible"] > 0] < 1.0 / 255.0).sum() > 100
    tiles, gids, ranges = oracle.tile_lists(p)
    nv, ni, ovf = frame.status()
    gt = frame.buffer(gsmi.BUF_INST_TILE).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    ge = frame.buffer(gsmi.BUF_INST_ENTRY).cpu().numpy()[:ni].view(np.uint32).astype(np.int64)
    gr = frame.buffer(gsmi.BUF_RANGES).cpu().numpy().view(np.uint32).reshape(-1, 2)
    nflag = _compare_lists(p, gt, ge, tiles, gids)
    _check_ranges_partition(gr, gt)
    if nflag == 0:
        assert ni == tiles.size and nv == int((p["visible"] > 0).sum())
        np.testing.assert_array_equal(_norm_ranges(gr), _norm_ranges(ranges))


@pytest.mark.parametrize("name", list(SCENES))
def test_3sigma_render_and_backward_match_oracle(name):
    sc = SCENES[name]
    cam = sc.cameras[0]
    frame, flat, params, cams_dev, opts = gpu_forward(sc, [cam], _opts(sc))
    p = oracle.project(sc, cam, footprint="3sigma")
    ref, Tref, nref, margin = oracle.render_image(p, sc.bg)
    img = flat.view(3, cam.height, cam.width).cpu().numpy()
    T = frame.buffer(gsmi.BUF_T_FINAL, torch.float32).cpu().numpy().reshape(cam.height, cam.width)
    nc = frame.buffer(gsmi.BUF_N_COMPOSITED).cpu().numpy().view(np.uint32).reshape(cam.height,
                                                                                 cam.width)
    good = margin > MARGIN
    assert good.mean() > 0.99
    scale = np.abs(ref) + np.abs(np.asarray(sc.bg, np.float64))[:, None, None]
    assert_close_scaled(img[:, good], ref[:, good], scale[:, good], what="image")
    assert_close_scaled(T[good], Tref[good], np.abs(Tref[good]), what="T_final")
    np.testing.assert_array_equal(nc[good], nref[good])
    # the adjoint
    rng = np.random.default_rng(6)
    dL = rng.standard_normal((3, cam.height, cam.width)) * 1e-3
    dL[:, ~good] = 0.0
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


def test_the_footprints_differ_only_where_the_square_cuts_the_ellipse():
    sc = SCENES["large_300_70x45_sh1"]
    cam = sc.cameras[0]
    _, a, *_ = gpu_forward(sc, [cam], _opts(sc, False))
    _, b, *_ = gpu_forward(sc, [cam], _opts(sc, True))
    a = a.view(3, cam.height, cam.width).cpu().numpy()
    b = b.view(3, cam.height, cam.width).cpu().numpy()
    pe = oracle.project(sc, cam)
    p3 = oracle.project(sc, cam, footprint="3sigma")
    re = oracle.render_image(pe, sc.bg)[0]
    r3 = oracle.render_image(p3, sc.bg)[0]
    differ = np.abs(re - r3).max(axis=0) > 1e-6
    assert differ.any()
    # the GPU images differ at those pixels, as the oracle's do
    assert (np.abs(a - b).max(axis=0)[differ] > 0).all()
