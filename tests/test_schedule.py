"""Coarse-to-fine schedule and global-to-local policy (Methodology, Eqs. 4-6):
the oracle's resampling and energies pinned to closed forms, the product's
schedule against the oracle, and the phase logic."""
import math

import numpy as np
import pytest
import torch

from oracle import schedule as ref
from paper_2507_20239_amd import gsmi, schedule


def _smooth_images(seed, n=3, H=96, W=128):
    rng = np.random.default_rng(seed)
    ys, xs = np.mgrid[0:H, 0:W]
    out = []
    for _ in range(n):
        img = np.zeros((3, H, W))
        for _ in range(12):
            cx, cy = rng.uniform(0, W), rng.uniform(0, H)
            s = rng.uniform(1.5, 20.0)
            col = rng.uniform(0, 1, 3)
            img += col[:, None, None] * np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / (2 * s * s))
        img += 0.05 * rng.standard_normal(img.shape)
        out.append(img)
    return out


# ---------------------------------------------------------------------------
# oracle pins
# ---------------------------------------------------------------------------
def test_oracle_downscale_identity_constant_and_ramp():
    rng = np.random.default_rng(0)
    img = rng.uniform(0, 1, (3, 40, 56))
    np.testing.assert_array_equal(ref.downscale(img, 1), img)
    c = np.full((3, 40, 56), 0.37)
    for r in (2, 3, 5):
        np.testing.assert_allclose(ref.downscale(c, r), 0.37, rtol=1e-14)
    # a linear ramp is reproduced exactly at the output pixel centres away from the border
    ramp = np.broadcast_to(np.arange(64, dtype=np.float64)[None, None, :] * 0.25, (1, 8, 64))
    out = ref.downscale(ramp, 4)                       # 2 x 16
    centres = (np.arange(16) + 0.5) * 4 - 0.5          # input-index coordinate of each centre
    np.testing.assert_allclose(out[0, 0, 1:-1], 0.25 * centres[1:-1], rtol=1e-12)


def test_oracle_energy_closed_forms():
    H, W = 64, 64
    c = np.full((3, H, W), 0.5)
    ratios = ref.energy_ratios([c], 8)
    for r, q in enumerate(ratios, start=1):
        h, w = round(H / r), round(W / r)
        assert q == pytest.approx(h * w * r * r / (H * W), rel=1e-12)
    # one cosine along x at frequency k: two DFT bins of magnitude H W / 2 per channel
    k = 3
    xs = np.arange(W)
    cos = np.broadcast_to(np.cos(2 * math.pi * k * xs / W)[None, None, :], (2, H, W))
    assert ref.energy(cos) == pytest.approx(2 * H * W, rel=1e-9)
    # white noise loses energy under antialiased downscaling
    noise = np.random.default_rng(1).standard_normal((3, 128, 128))
    q = ref.energy_ratios([noise], 4)
    assert q[0] == 1.0 and q[1] < 1.0 and q[2] < q[1] and q[3] < q[2]


# ---------------------------------------------------------------------------
# the product against the oracle
# ---------------------------------------------------------------------------
def test_downscale_matches_oracle():
    img = _smooth_images(2, n=1)[0]
    t = torch.from_numpy(img)
    for r in (2, 3, 4, 7):
        np.testing.assert_allclose(schedule.downscale(t, r).numpy(), ref.downscale(img, r),
                                   rtol=1e-9, atol=1e-12)


def test_energy_ratios_and_boundaries_match_oracle():
    imgs = _smooth_images(3)
    got = schedule.energy_ratios([torch.from_numpy(i) for i in imgs], 8)
    want = ref.energy_ratios(imgs, 8)
    np.testing.assert_allclose(got, want, rtol=1e-9)
    assert got[0] == 1.0
    assert schedule.c2f_boundaries(got, 25000) == ref.boundaries(imgs, 8, 25000)


# ---------------------------------------------------------------------------
# phase logic
# ---------------------------------------------------------------------------
def test_c2f_schedule_runs_coarsest_first():
    s = schedule.C2FSchedule([1000, 600, 300, 300, 100])      # T_1..T_5
    # scale 5 over [0, 100), 4 over [100, 300), 3 empty, 2 over [300, 600), then full
    assert [s.resolution(i) for i in (0, 99)] == [5, 5]
    assert [s.resolution(i) for i in (100, 299)] == [4, 4]
    assert [s.resolution(i) for i in (300, 599)] == [2, 2]
    assert [s.resolution(i) for i in (600, 1000, 29999)] == [1, 1, 1]
    assert s.full_resolution_from() == 600
    # a scale whose T_r is below a coarser one's starts where the coarser ended
    s2 = schedule.C2FSchedule([800, 200, 500])
    assert [s2.resolution(i) for i in (0, 499, 500, 799)] == [3, 3, 1, 1]


def test_global_to_local_policy():
    s = schedule.C2FSchedule([25000, 9000, 6000, 4000])
    p = schedule.GlobalToLocal(s)
    assert p.global_phase(8999) and not p.allow_clone(8999)
    assert p.allow_clone(9000)
    assert p.densify_now(500) and p.densify_now(24900) and not p.densify_now(25000)
    assert not p.densify_now(450) and not p.densify_now(501)
    assert p.opacity_reset_now(3000) and p.opacity_reset_now(24000) and not p.opacity_reset_now(0)
    assert p.position_lr(0) == p.position_lr(8999) == p.lr_position_init
    assert p.position_lr(30000) == pytest.approx(p.lr_position_final)
    assert p.position_lr(9000) > p.position_lr(20000) > p.position_lr(30000)
    g, ls, lo = p.thresholds(4.4)
    assert ls == pytest.approx(math.log(0.044)) and lo == pytest.approx(math.log(0.05 / 0.95))


def test_densification_strategies():
    s = schedule.C2FSchedule([25000, 9000, 6000, 4000])
    g2l = schedule.GlobalToLocal(s)
    assert g2l.densify_mode(8999) == gsmi.DENSIFY_SPLIT_LARGE
    assert g2l.densify_mode(9000) == gsmi.DENSIFY_ADAPTIVE
    for strategy, mode in (("3dgs", gsmi.DENSIFY_ADAPTIVE), ("split_only", gsmi.DENSIFY_SPLIT_ONLY),
                           ("clone_only", gsmi.DENSIFY_CLONE_ONLY)):
        p = schedule.GlobalToLocal(s, strategy=strategy)
        assert p.densify_mode(0) == p.densify_mode(20000) == mode
        assert p.allow_clone(0) == (strategy != "split_only")
    with pytest.raises(ValueError):
        schedule.GlobalToLocal(s, strategy="clone-only")
