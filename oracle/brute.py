"""Dense brute-force reference in float64 PyTorch (CPU) with autograd.

TEST INFRASTRUCTURE ONLY.  It exists to pin the C oracle's hand-written
adjoint: every pixel evaluates every Gaussian as dense tensors, the per-pixel
front-to-back product is a cumulative product over the globally depth-ordered
Gaussians, and gradients come from torch autograd instead of a hand-derived
chain rule.  The spherical harmonics are evaluated here from spherical angles
with the textbook associated Legendre functions (Condon-Shortley phase), not
from the polynomial form the C oracle uses.  Only for tiny scenes (memory is
pixels x Gaussians).

Passages: Eq. 1 (Gaussian, Sigma = R S S^T R^T), Sigma' = J W Sigma W^T J^T,
Eq. 2 (compositing) of "Decomposing Densification in Gaussian Splatting".
"""
from __future__ import annotations

import math

import numpy as np
import torch

ALPHA_MAX = float(np.float32(0.99))
ALPHA_MIN = float(np.float32(1.0 / 255.0))
T_MIN = float(np.float32(1e-4))
DILATION = float(np.float32(0.3))


def _assoc_legendre(l, m, x, s):
    """P_l^m(cos th) with the Condon-Shortley phase, x = cos th, s = sin th."""
    table = {
        (0, 0): lambda: torch.ones_like(x),
        (1, 0): lambda: x,
        (1, 1): lambda: -s,
        (2, 0): lambda: 0.5 * (3 * x * x - 1),
        (2, 1): lambda: -3 * x * s,
        (2, 2): lambda: 3 * s * s,
        (3, 0): lambda: 0.5 * (5 * x ** 3 - 3 * x),
        (3, 1): lambda: -1.5 * (5 * x * x - 1) * s,
        (3, 2): lambda: 15 * x * s * s,
        (3, 3): lambda: -15 * s ** 3,
    }
    return table[(l, m)]()


def sh_basis_angles(deg, d):
    """Y[k] (k = l^2 + l + m) at unit directions d (N, 3), via (theta, phi)."""
    theta = torch.acos(torch.clamp(d[:, 2], -1.0, 1.0))
    phi = torch.atan2(d[:, 1], d[:, 0])
    x = torch.cos(theta)
    s = torch.sin(theta)
    out = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) /
                          math.factorial(l + am))
            P = _assoc_legendre(l, am, x, s)
            if m == 0:
                out.append(K * P)
            elif m > 0:
                out.append(math.sqrt(2) * K * P * torch.cos(am * phi))
            else:
                out.append(math.sqrt(2) * K * P * torch.sin(am * phi))
    return torch.stack(out, 0)  # (K, N)


def _quat_rot(q):
    w, x, y, z = q
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]),
    ])  # (3, 3, N)


def render_dense(means, log_scales, quats, logits, sh, deg, cam, bg=(0, 0, 0), near=0.2,
                 depth_key=None):
    """Differentiable dense render of one view.  Tensors are float64, SoA as
    in the GPU library.  `depth_key` (uint32 numpy, FP32 depth bits) fixes the
    depth order; when None it is derived from the camera depth."""
    W, H = cam.width, cam.height
    Rw = torch.tensor(cam.R, dtype=torch.float64)
    tw = torch.tensor(cam.t, dtype=torch.float64)
    fx, fy, cx, cy = cam.fx, cam.fy, cam.cx, cam.cy
    s = torch.exp(log_scales)
    qn = quats / torch.linalg.norm(quats, dim=0, keepdim=True)
    o = torch.sigmoid(logits)
    R = _quat_rot(qn).permute(2, 0, 1)  # (N, 3, 3)
    M = R * s.T[:, None, :]
    Sigma = M @ M.transpose(1, 2)
    t = (Rw @ means) + tw[:, None]  # (3, N)
    tz = t[2]
    culled = ~(tz > near)
    limx = 1.3 * 0.5 * W / fx
    limy = 1.3 * 0.5 * H / fy
    xt = torch.clamp(t[0] / tz, -limx, limx)
    yt = torch.clamp(t[1] / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * xt / tz]),
                     torch.stack([zero, fy / tz, -fy * yt / tz])]).permute(2, 0, 1)  # (N,2,3)
    T = J @ Rw
    cov = T @ Sigma @ T.transpose(1, 2) + DILATION * torch.eye(2, dtype=torch.float64)
    det = cov[:, 0, 0] * cov[:, 1, 1] - cov[:, 0, 1] * cov[:, 1, 0]
    ca = cov[:, 1, 1] / det
    cb = -0.5 * (cov[:, 0, 1] + cov[:, 1, 0]) / det
    cc = cov[:, 0, 0] / det
    mx = fx * t[0] / tz + cx
    my = fy * t[1] / tz + cy
    centre = -(Rw.T @ tw)
    dvec = means - centre[:, None]
    dirs = (dvec / torch.linalg.norm(dvec, dim=0, keepdim=True)).T
    Y = sh_basis_angles(deg, dirs)  # (K, N)
    rgb = torch.clamp_min(torch.einsum("kn,kcn->cn", Y, sh) + 0.5, 0.0)  # (3, N)

    if depth_key is None:
        depth_key = tz.detach().numpy().astype(np.float32).view(np.uint32)
    order = np.lexsort((np.arange(tz.shape[0]), depth_key))
    order = order[~culled.numpy()[order]]
    ot = torch.as_tensor(order)

    ys, xs = torch.meshgrid(torch.arange(H, dtype=torch.float64),
                            torch.arange(W, dtype=torch.float64), indexing="ij")
    px = (xs.reshape(-1) + 0.5)[:, None]
    py = (ys.reshape(-1) + 0.5)[:, None]
    dx = px - mx[ot][None, :]
    dy = py - my[ot][None, :]
    power = -0.5 * (ca[ot] * dx * dx + cc[ot] * dy * dy) - cb[ot] * dx * dy
    G = torch.exp(power)
    raw = o[ot][None, :] * G
    cand = (raw >= ALPHA_MIN).detach()
    alpha = torch.clamp(raw, max=ALPHA_MAX)
    a0 = torch.where(cand, alpha, torch.zeros_like(alpha)).detach()
    T_excl = torch.cumprod(torch.cat([torch.ones_like(a0[:, :1]), 1 - a0[:, :-1]], 1), 1)
    stop = cand & (T_excl * (1 - a0) < T_MIN)
    after = torch.cumsum(stop.to(torch.int64), 1) > 0
    used = cand & ~after
    a = torch.where(used, alpha, torch.zeros_like(alpha))
    Tx = torch.cumprod(torch.cat([torch.ones_like(a[:, :1]), 1 - a[:, :-1]], 1), 1)
    Tf = torch.prod(1 - a, 1)
    w = a * Tx
    bgt = torch.tensor(bg, dtype=torch.float64)
    C = w @ rgb[:, ot].T + Tf[:, None] * bgt[None, :]  # (P, 3)
    return C.T.reshape(3, H, W), Tf.reshape(H, W)


def scene_tensors(scene):
    names = ["means", "log_scales", "quats", "opacity_logits", "sh"]
    return {k: torch.tensor(np.asarray(getattr(scene, k), np.float64), requires_grad=True)
            for k in names}
