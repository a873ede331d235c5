"""Reference for the photometric loss of Eq. 3 with its D-SSIM term,
L = (1 - lambda) mean |I - T| + lambda (1 - mean SSIM(I, T)), in FP64 with
plain torch CPU operations; the gradient by torch autograd.  TEST
INFRASTRUCTURE ONLY.  SSIM per channel with an 11 x 11 Gaussian window
(standard deviation 1.5, normalised), zero padding, C1 = 0.01^2,
C2 = 0.03^2 (the 3DGS convention the paper trains with)."""
import math

import numpy as np
import torch
import torch.nn.functional as F


def window(radius=5, sigma=1.5):
    g = np.array([math.exp(-((k - radius) ** 2) / (2 * sigma * sigma)) for k in range(2 * radius + 1)])
    return g / g.sum()


def ssim_map(img, tgt):
    """SSIM at every pixel of [C, H, W] tensors (FP64)."""
    C = img.shape[0]
    g = torch.tensor(window(), dtype=torch.float64)
    w2 = torch.outer(g, g)[None, None].repeat(C, 1, 1, 1)

    def filt(x):
        return F.conv2d(x[None], w2, padding=5, groups=C)[0]

    mu, nu = filt(img), filt(tgt)
    sxx = filt(img * img) - mu * mu
    syy = filt(tgt * tgt) - nu * nu
    sxy = filt(img * tgt) - mu * nu
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    return ((2 * mu * nu + c1) * (2 * sxy + c2)) / ((mu * mu + nu * nu + c1) * (sxx + syy + c2))


def loss_and_grad(img, tgt, lam=0.2):
    """(L, dL/dI) for [C, H, W] arrays."""
    x = torch.tensor(np.asarray(img, np.float64), requires_grad=True)
    y = torch.tensor(np.asarray(tgt, np.float64))
    L = (1 - lam) * (x - y).abs().mean() + lam * (1 - ssim_map(x, y).mean())
    L.backward()
    return float(L), x.grad.numpy()
