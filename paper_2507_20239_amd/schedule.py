"""Training schedule of the paper's method around the rasterizer: the
energy-guided coarse-to-fine resolution schedule (Methodology, Coarse-to-fine
multi-resolution densification, Eqs. 4-6) and the global-to-local
densification phases it delimits (Methodology, Global-to-local framework),
with the densification cadence, opacity reset and adaptive opacity pruning
parameters (Preliminary; Adaptive Opacity Pruning; Experiments,
implementation details).

Host logic that runs once per scene (the energies) or once per iteration (a
few comparisons); the image work is torch library calls (FFT, antialiased
bilinear resampling).  Readings where the paper is silent:
  - E_r is averaged over the training images; the FFT magnitude is summed
    over colour channels; the downscaled size is round(H / r) x round(W / r);
  - T_{K+1} = 0, and a scale whose interval [T_{r+1}, T_r) is empty or
    overlaps a coarser one starts where the coarser one ended: scale r runs
    over [e_{r+1}, e_r) with e_r = max(T_r, e_{r+1});
  - the global (split-only) phase is the time spent below full resolution,
    i.e. iterations before e_2; clones are allowed from then on;
  - the position learning rate stays at its initial value below full
    resolution and decays exponentially to its final value afterwards.
"""
from __future__ import annotations

import dataclasses
import math

import torch
import torch.nn.functional as F

from . import gsmi


def downscale(image: torch.Tensor, r: int) -> torch.Tensor:
    """D_r (Eq. 4): bilinear resampling with antialiasing by 1/r; [C, H, W]."""
    if r == 1:
        return image
    C, H, W = image.shape
    size = (max(1, int(round(H / r))), max(1, int(round(W / r))))
    return F.interpolate(image[None], size=size, mode="bilinear", antialias=True,
                         align_corners=False)[0]


def energy(image: torch.Tensor) -> float:
    """||E(I)||_1: the L1 norm of the 2D FFT magnitude, summed over channels."""
    spec = torch.fft.fft2(image.to(torch.float64))
    return float(spec.abs().sum())


def energy_ratios(images, K: int) -> list:
    """E_r / E_1 for r = 1..K with E_r = ||E(I_r)||_1 r^2 (Eq. 5), averaged
    over the images."""
    tot = [0.0] * (K + 1)
    for img in images:
        img = torch.as_tensor(img)
        for r in range(1, K + 1):
            tot[r] += energy(downscale(img, r)) * r * r
    return [tot[r] / tot[1] for r in range(1, K + 1)]


def c2f_boundaries(ratios, t_densify: int) -> list:
    """T_r = Round((E_r / E_1) T_densify) for r = 1..K (Eq. 6)."""
    return [int(round(q * t_densify)) for q in ratios]


@dataclasses.dataclass
class C2FSchedule:
    """Scale r is trained over [e_{r+1}, e_r), coarsest first; full resolution
    from e_2 on."""
    t_r: list               # T_1..T_K

    def __post_init__(self):
        K = len(self.t_r)
        self.ends = [0] * (K + 2)          # ends[r] = e_r, ends[K + 1] = 0
        for r in range(K, 0, -1):
            self.ends[r] = max(self.t_r[r - 1], self.ends[r + 1])

    @classmethod
    def from_images(cls, images, K: int = 8, t_densify: int = 25000):
        return cls(c2f_boundaries(energy_ratios(images, K), t_densify))

    @property
    def K(self) -> int:
        return len(self.t_r)

    def resolution(self, it: int) -> int:
        """Downscale factor r of iteration it."""
        for r in range(self.K, 1, -1):
            if self.ends[r + 1] <= it < self.ends[r]:
                return r
        return 1

    def full_resolution_from(self) -> int:
        return self.ends[2] if self.K >= 2 else 0


@dataclasses.dataclass
class GlobalToLocal:
    """Densification policy.  Defaults: 3DGS cadence (every 100 iterations from
    500, opacity reset every 3000) extended to T_densify = 25000, adaptive
    pruning p = 0.03, tau_u = 0.05, split threshold 2e-4 on the view-space
    gradient, scale threshold 1% of the scene extent.

    strategy picks what a selected Gaussian becomes: "g2l" (the paper's
    global-to-local framework: split-only while below full resolution, the
    3DGS rule after), "3dgs" (the 3DGS rule throughout), "split_only" or
    "clone_only" (the single-operation variants of the Gaussian distribution
    comparison)."""
    schedule: C2FSchedule
    t_densify: int = 25000
    densify_from: int = 500
    interval: int = 100
    opacity_reset_every: int = 3000
    grad_threshold: float = 2e-4
    scale_ratio: float = 0.01
    prune_ratio: float = 0.03
    prune_upper: float = 0.05
    lr_position_init: float = 1.6e-4
    lr_position_final: float = 1.6e-6
    total_iterations: int = 30000
    strategy: str = "g2l"

    STRATEGIES = ("g2l", "3dgs", "split_only", "clone_only")

    def __post_init__(self):
        if self.strategy not in self.STRATEGIES:
            raise ValueError("strategy must be one of %s" % (self.STRATEGIES,))

    def global_phase(self, it: int) -> bool:
        """Split only (clones suppressed) while training below full resolution."""
        return it < self.schedule.full_resolution_from()

    def allow_clone(self, it: int) -> bool:
        return self.densify_mode(it) in (gsmi.DENSIFY_ADAPTIVE, gsmi.DENSIFY_CLONE_ONLY)

    def densify_mode(self, it: int) -> int:
        """The gsmi.DENSIFY_* mode of the selection at iteration it."""
        if self.strategy == "g2l":
            return gsmi.DENSIFY_SPLIT_LARGE if self.global_phase(it) else gsmi.DENSIFY_ADAPTIVE
        return {"3dgs": gsmi.DENSIFY_ADAPTIVE, "split_only": gsmi.DENSIFY_SPLIT_ONLY,
                "clone_only": gsmi.DENSIFY_CLONE_ONLY}[self.strategy]

    def densify_now(self, it: int) -> bool:
        return self.densify_from <= it < self.t_densify and it % self.interval == 0

    def opacity_reset_now(self, it: int) -> bool:
        return 0 < it < self.t_densify and it % self.opacity_reset_every == 0

    def position_lr(self, it: int, extent: float = 1.0) -> float:
        t0 = self.schedule.full_resolution_from()
        if it < t0:
            return self.lr_position_init * extent
        span = max(1, self.total_iterations - t0)
        s = min(1.0, (it - t0) / span)
        return extent * math.exp((1 - s) * math.log(self.lr_position_init) +
                                 s * math.log(self.lr_position_final))

    def thresholds(self, extent: float):
        """(grad threshold, ln(rho E), logit-space upper prune limit) as floats."""
        return (self.grad_threshold, math.log(self.scale_ratio * extent),
                math.log(self.prune_upper / (1.0 - self.prune_upper)))
