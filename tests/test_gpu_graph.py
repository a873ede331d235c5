"""The captured training step (project -> render -> L1 -> render backward ->
project backward with the statistic) replayed several times, with eager work
and synchronisations between the replays, against the same step run eagerly
on separate buffers.  Images and loss gradients are deterministic (no atomics)
and must be bit-identical; splat gradients, parameter gradients, the loss and
the statistic are summed with FP32 atomics in an unspecified order and are
compared to 1e-5 of their scale."""
import numpy as np
import pytest
import torch

from paper_2507_20239_amd import gsmi, synth
from parity_util import dev, params_of

pytestmark = pytest.mark.gpu


class _Bufs:
    def __init__(self, sc, cams, opts, cap):
        self.frame = gsmi.Frame(sc.n, [(c.width, c.height) for c in cams], cap, dev())
        self.images = torch.empty(self.frame.image_numel(), device=dev())
        self.loss = torch.zeros(1, device=dev())
        self.dL = torch.empty_like(self.images)
        self.acc = torch.zeros(sc.n, device=dev())
        self.den = torch.zeros(sc.n, device=dev())


def _close(a, b, what):
    a = a.detach().cpu().numpy().astype(np.float64)
    b = b.detach().cpu().numpy().astype(np.float64)
    scale = max(np.abs(b).max(), 1e-30)
    np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-5 * scale, err_msg=what)


@pytest.mark.parametrize("persistent", [0, 512])
def test_graph_replays_match_eager_steps(persistent):
    sc = synth.random_scene(41, 3000, 160, 120, sh_degree=3, n_views=3, log_scale=(-2.4, 0.5))
    cams = [sc.cameras[0], sc.cameras[1].scaled(2), sc.cameras[2]]
    opts = gsmi.raster_opts(persistent_blocks=persistent)
    params = params_of(sc)
    cams_dev = gsmi.cameras_to_device(cams, dev())
    cap = 1 << 20
    ge, gg = _Bufs(sc, cams, opts, cap), _Bufs(sc, cams, opts, cap)
    targets = torch.rand(ge.frame.image_numel(), device=dev(), generator=None)
    scale = 1.0 / targets.numel()
    grads_e, grads_g = gsmi.empty_grads(params), gsmi.empty_grads(params)
    graph = gsmi.StepGraph(gg.frame, params, sc.sh_degree, cams_dev, opts, gg.images, targets,
                           scale, gg.loss, gg.dL, grads_g, gg.acc, gg.den)
    for replay in range(4):
        graph.launch()
        torch.cuda.synchronize()
        # the eager step, on its own frame and buffers
        f = ge.frame
        f.project(params, sc.sh_degree, cams_dev, opts)
        f.render(opts, ge.images)
        ge.loss.zero_()
        gsmi.l1_loss_grad(ge.images, targets, scale, ge.loss, ge.dL)
        f.render_backward(opts, ge.dL)
        f.project_backward(params, sc.sh_degree, cams_dev, opts, grads_e, ge.acc, ge.den)
        torch.cuda.synchronize()
        assert torch.equal(gg.images, ge.images), replay
        assert torch.equal(gg.dL, ge.dL), replay
        _close(gg.loss, ge.loss, "loss")
        sge = f.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32)
        sgg = gg.frame.buffer(gsmi.BUF_SPLAT_GRAD, torch.float32)
        tt = f.buffer(gsmi.BUF_TILES_TOUCHED) > 0
        assert torch.equal(tt, gg.frame.buffer(gsmi.BUF_TILES_TOUCHED) > 0)
        _close(sgg.view(-1, 9)[tt], sge.view(-1, 9)[tt], "splat gradients")
        for k in gsmi.PARAM_NAMES:
            _close(grads_g[k], grads_e[k], k)
        _close(gg.acc, ge.acc, "statistic")
        assert torch.equal(gg.den, ge.den)
        assert 0 < float(gg.den.max()) <= 3 * (replay + 1)
