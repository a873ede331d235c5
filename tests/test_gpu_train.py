"""The training driver on a small synthetic scene: the coarse-to-fine
schedule moves from coarse to full resolution, the global phase densifies by
splitting only, clones appear in the local phase, opacities are reset, the
adaptive threshold prunes, the full-resolution loss falls and the lineage
attributes follow every compaction; the single-operation strategies densify
with one operation only."""
import numpy as np
import pytest
import torch

from paper_2507_20239_amd import gsmi, schedule, synth
from paper_2507_20239_amd.train import Trainer
from parity_util import dev, params_of

pytestmark = pytest.mark.gpu


def _render(params, sh_degree, cam):
    frame = gsmi.Frame(params["means"].shape[-1], [(cam.width, cam.height)], 1 << 20, dev())
    opts = gsmi.raster_opts()
    frame.project(params, sh_degree, gsmi.cameras_to_device([cam], dev()), opts)
    img = frame.render(opts)
    torch.cuda.synchronize()
    return img.view(3, cam.height, cam.width).clone()


def _full_res_loss(tr, cams, targets):
    tot = 0.0
    for cam, t in zip(cams, targets):
        img = _render(tr.p, tr.sh_degree, cam)
        loss, _ = gsmi.ssim_loss_grad(img, t.to(dev()), 0.2)
        tot += float(loss)
    return tot / len(cams)


def _scene():
    gt = synth.random_scene(61, 3000, 128, 96, sh_degree=1, n_views=4, log_scale=(-3.2, 0.4),
                            logit=(1.0, 1.0))
    cams = gt.cameras
    targets = [_render(params_of(gt), gt.sh_degree, c).cpu() for c in cams]
    init = synth.random_scene(62, 400, 128, 96, sh_degree=1, log_scale=(-2.5, 0.3), logit=(0.0, 0.5))
    return cams, targets, init


def _origins_are_initial_means(tr, init):
    start = {tuple(c) for c in np.asarray(init.means, np.float32).T.tolist()}
    origin = tr.lineage["origin"].cpu().numpy()
    assert origin.shape == (3, tr.n)
    assert all(tuple(c) in start for c in origin.T.tolist())


def test_global_to_local_training_on_a_synthetic_scene():
    cams, targets, init = _scene()
    sched = schedule.C2FSchedule.from_images(targets, K=4, t_densify=450)
    policy = schedule.GlobalToLocal(sched, t_densify=450, densify_from=50, interval=50,
                                    opacity_reset_every=150, grad_threshold=2e-4,
                                    total_iterations=500)
    tr = Trainer(params_of(init), init.sh_degree, cams, targets, policy, extent=1.0, seed=3,
                 device=dev(), lineage=True)
    before = _full_res_loss(tr, cams, targets)
    for it in range(500):
        tr.step(it)
    after = _full_res_loss(tr, cams, targets)
    print("schedule", sched.t_r, "full res from", sched.full_resolution_from(), flush=True)
    print("loss", before, "->", after, "n", 400, "->", tr.n, flush=True)
    for row in tr.densify_log:
        print("densify", row, flush=True)
    res = [h[3] for h in tr.history]
    assert res[0] == max(res) and res[-1] == 1 and all(a >= b for a, b in zip(res, res[1:]))
    glob = [d for d in tr.densify_log if d[6] == gsmi.DENSIFY_SPLIT_LARGE]
    loc = [d for d in tr.densify_log if d[6] == gsmi.DENSIFY_ADAPTIVE]
    assert len(glob) + len(loc) == len(tr.densify_log)
    assert all(d[3] == 0 for d in glob)              # split only in the global phase
    assert any(d[4] > 0 for d in glob) and loc and any(d[3] > 0 for d in loc)
    assert after < 0.8 * before
    # lineage: every original position is an initial mean; counts are whole numbers;
    # the categories cover every Gaussian.  Clones only start in the local phase,
    # mostly from Gaussians that split before (the equal category).
    _origins_are_initial_means(tr, init)
    ns = tr.lineage["splits"].cpu().numpy()
    nc = tr.lineage["clones"].cpu().numpy()
    assert (ns == np.round(ns)).all() and (nc == np.round(nc)).all() and ns.min() >= 0
    summary = tr.lineage_summary()
    print("lineage", summary, flush=True)
    assert sum(v[0] for v in summary.values()) == tr.n
    assert summary["split"][0] > 0 and summary["equal"][0] > 0
    assert summary["clone"][0] == int(((nc > ns) & (nc > 0)).sum())


@pytest.mark.parametrize("strategy", ["split_only", "clone_only"])
def test_single_operation_strategies(strategy):
    cams, targets, init = _scene()
    sched = schedule.C2FSchedule([200, 100])
    policy = schedule.GlobalToLocal(sched, t_densify=200, densify_from=50, interval=50,
                                    opacity_reset_every=1000, grad_threshold=2e-4,
                                    total_iterations=200, strategy=strategy)
    tr = Trainer(params_of(init), init.sh_degree, cams, targets, policy, extent=1.0, seed=5,
                 device=dev(), lineage=True)
    for it in range(200):
        tr.step(it)
    for row in tr.densify_log:
        print("densify", row, flush=True)
    assert len(tr.densify_log) == 3
    col_used, col_unused = (4, 3) if strategy == "split_only" else (3, 4)
    assert all(d[col_unused] == 0 for d in tr.densify_log)
    assert any(d[col_used] > 0 for d in tr.densify_log)
    _origins_are_initial_means(tr, init)
    unused = tr.lineage["clones" if strategy == "split_only" else "splits"]
    used = tr.lineage["splits" if strategy == "split_only" else "clones"]
    assert not unused.any() and used.any()
