"""Reference for the coarse-to-fine resolution schedule (Methodology,
Coarse-to-fine multi-resolution densification, Eqs. 4-6), written from the
definitions with numpy only.  TEST INFRASTRUCTURE ONLY (tests and the
benchmark's CPU leg import it; the product never does).

  D_r(I): bilinear resampling by 1/r with antialiasing -- each output sample
          at centre c (in input pixel units, pixel j spans [j, j+1)) is the
          normalised triangle-weighted average of the input samples,
          weight(j) = max(0, 1 - |j + 1/2 - c| / s), s = input / output size
          (the stretched bilinear kernel), separable over rows and columns;
  E(I)  = |F(I)|, the 2D DFT magnitude, summed over channels;
  E_r   = ||E(D_r(I))||_1 r^2, averaged over images;
  T_r   = Round(E_r / E_1 T_densify).
"""
import numpy as np


def _resample_axis(a: np.ndarray, axis: int, out: int) -> np.ndarray:
    n = a.shape[axis]
    s = n / out
    c = (np.arange(out) + 0.5) * s                      # output centres
    j = np.arange(n) + 0.5                              # input centres
    w = np.maximum(0.0, 1.0 - np.abs(j[None, :] - c[:, None]) / s)
    w /= w.sum(1, keepdims=True)
    return np.moveaxis(np.tensordot(w, np.moveaxis(a, axis, 0), axes=(1, 0)), 0, axis)


def downscale(image, r: int) -> np.ndarray:
    img = np.asarray(image, np.float64)
    if r == 1:
        return img
    C, H, W = img.shape
    h, w = max(1, int(round(H / r))), max(1, int(round(W / r)))
    return _resample_axis(_resample_axis(img, 1, h), 2, w)


def energy(image) -> float:
    img = np.asarray(image, np.float64)
    return float(sum(np.abs(np.fft.fft2(img[c])).sum() for c in range(img.shape[0])))


def energy_ratios(images, K: int) -> list:
    tot = np.zeros(K + 1)
    for img in images:
        for r in range(1, K + 1):
            tot[r] += energy(downscale(img, r)) * r * r
    return [tot[r] / tot[1] for r in range(1, K + 1)]


def boundaries(images, K: int, t_densify: int) -> list:
    return [int(round(q * t_densify)) for q in energy_ratios(images, K)]
