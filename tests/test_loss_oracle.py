"""Pins of the loss oracle (Eq. 3 with D-SSIM): the window sums to one, SSIM
is 1 for identical images, the interior SSIM of two constant images has its
closed form, the filtered statistics match explicit window sums, and the
autograd gradient matches central differences."""
import numpy as np
import pytest
import torch

from oracle import loss as ref


def test_window_and_identity():
    g = ref.window()
    assert g.sum() == pytest.approx(1.0, abs=1e-15) and g.argmax() == 5
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.uniform(0, 1, (3, 20, 24)))
    np.testing.assert_allclose(ref.ssim_map(x, x).numpy(), 1.0, rtol=1e-12)
    L, g = ref.loss_and_grad(x.numpy(), x.numpy())
    assert L == pytest.approx(0.0, abs=1e-12)


def test_constant_images_closed_form_in_the_interior():
    c, d = 0.3, 0.7
    s = ref.ssim_map(torch.full((1, 30, 30), c, dtype=torch.float64),
                     torch.full((1, 30, 30), d, dtype=torch.float64)).numpy()[0]
    c1 = 0.01 ** 2
    want = (2 * c * d + c1) / (c * c + d * d + c1)
    np.testing.assert_allclose(s[5:-5, 5:-5], want, rtol=1e-12)


def test_statistics_match_explicit_window_sums():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (2, 17, 19))
    y = rng.uniform(0, 1, (2, 17, 19))
    s = ref.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    g = ref.window()
    W2 = np.outer(g, g)
    xp = np.pad(x, ((0, 0), (5, 5), (5, 5)))
    yp = np.pad(y, ((0, 0), (5, 5), (5, 5)))
    for (ch, i, j) in [(0, 0, 0), (1, 8, 9), (0, 16, 18), (1, 3, 15)]:
        px, py = xp[ch, i:i + 11, j:j + 11], yp[ch, i:i + 11, j:j + 11]
        mu, nu = (W2 * px).sum(), (W2 * py).sum()
        sxx = (W2 * px * px).sum() - mu * mu
        syy = (W2 * py * py).sum() - nu * nu
        sxy = (W2 * px * py).sum() - mu * nu
        c1, c2 = 0.01 ** 2, 0.03 ** 2
        want = (2 * mu * nu + c1) * (2 * sxy + c2) / ((mu * mu + nu * nu + c1) * (sxx + syy + c2))
        assert s[ch, i, j] == pytest.approx(want, rel=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (3, 13, 14))
    y = rng.uniform(0, 1, (3, 13, 14))
    L, g = ref.loss_and_grad(x, y, lam=0.2)
    h = 1e-6
    for (c, i, j) in [(0, 0, 0), (1, 6, 7), (2, 12, 13), (0, 4, 11), (1, 11, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += h
        xm[c, i, j] -= h
        fd = (ref.loss_and_grad(xp, y)[0] - ref.loss_and_grad(xm, y)[0]) / (2 * h)
        assert g[c, i, j] == pytest.approx(fd, rel=1e-5, abs=1e-10)
