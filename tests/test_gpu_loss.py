"""The fused L1 + D-SSIM loss kernel (Eq. 3) against the FP64 oracle: the
loss value and its gradient w.r.t. the rendered image, on ragged and
full-size images."""
import numpy as np
import pytest
import torch

from oracle import loss as ref
from paper_2507_20239_amd import gsmi
from parity_util import dev

pytestmark = pytest.mark.gpu


def _images(kind, C, H, W, seed):
    rng = np.random.default_rng(seed)
    ys, xs = np.mgrid[0:H, 0:W]
    if kind == "noise":
        return rng.uniform(0, 1, (C, H, W)), rng.uniform(0, 1, (C, H, W))
    base = np.stack([0.5 + 0.4 * np.sin(xs / (7.0 + c) + ys / (11.0 + 2 * c)) for c in range(C)])
    if kind == "smooth":
        return base + 0.02 * rng.standard_normal((C, H, W)), base
    return base + 0.2 * rng.standard_normal((C, H, W)), base   # "noisy copy"


@pytest.mark.parametrize("kind,C,H,W", [("noise", 3, 37, 53), ("smooth", 3, 64, 80),
                                        ("noisy", 1, 16, 16), ("smooth", 3, 1040, 1600)])
def test_loss_and_gradient_match_oracle(kind, C, H, W):
    x, y = _images(kind, C, H, W, seed=H)
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    L_ref, g_ref = ref.loss_and_grad(x32.astype(np.float64), y32.astype(np.float64), lam=0.2)
    loss, grad = gsmi.ssim_loss_grad(torch.from_numpy(x32).to(dev()),
                                     torch.from_numpy(y32).to(dev()), 0.2)
    torch.cuda.synchronize()
    assert float(loss) == pytest.approx(L_ref, rel=2e-5, abs=1e-7)
    g = grad.cpu().numpy().astype(np.float64)
    err = np.abs(g - g_ref)
    scale = np.abs(g_ref).max()
    print(kind, C, H, W, "max err / max |g|", err.max() / scale, flush=True)
    assert (err <= 1e-4 * scale + 1e-3 * np.abs(g_ref)).all()
