"""Seeded synthetic inputs shaped like the paper's training workloads.

This module only draws numbers.  It holds none of the method's arithmetic
(no projection, no compositing, no densification); both the HIP path and the
FP64 oracle receive exactly the arrays produced here, so it is the one piece of
code they share.

Layouts (structure of arrays, FP32, Gaussian index fastest):
  means          [3][N]        world-space centres
  log_scales     [3][N]        log of the per-axis standard deviations
  quats          [4][N]        rotation quaternion (w, x, y, z), not necessarily unit
  opacity_logits [N]           opacity = sigmoid(logit)
  sh             [K][3][N]     real spherical-harmonic coefficients, K = (deg+1)^2
Cameras are world->camera rigid transforms in OpenCV axes (x right, y down,
z forward) with pinhole intrinsics in pixels.

The paper's datasets (MipNeRF-360, Deep Blending, Tanks & Temples) are not
available; these generators stand in for them with scene sizes bracketing the
paper's final Gaussian counts (Table 2: 0.87M-2.58M primitives).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# sqrt(pi): with a degree-0 colour  rgb = Y00 * f + 1/2  and Y00 = 1/(2 sqrt(pi)),
# a DC coefficient drawn from U(-sqrt(pi), sqrt(pi)) gives rgb ~ U(0, 1).
_DC_HALF_RANGE_FOR_UNIT_RGB = math.sqrt(math.pi)


@dataclasses.dataclass
class Camera:
    R: np.ndarray        # (3, 3) float64, world -> camera rotation (rows: right, down, forward)
    t: np.ndarray        # (3,) float64
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def __post_init__(self):
        # cameras travel to the GPU as FP32: keep exactly the FP32 values here too
        self.R = np.asarray(self.R, np.float32).astype(np.float64)
        self.t = np.asarray(self.t, np.float32).astype(np.float64)
        self.fx, self.fy = float(np.float32(self.fx)), float(np.float32(self.fy))
        self.cx, self.cy = float(np.float32(self.cx)), float(np.float32(self.cy))
        self.width, self.height = int(self.width), int(self.height)

    def scaled(self, r: int) -> "Camera":
        """The same pose rendered at 1/r resolution (coarse-to-fine level r)."""
        w = int(round(self.width / r))
        h = int(round(self.height / r))
        return Camera(self.R.copy(), self.t.copy(), self.fx / r, self.fy / r,
                      self.cx / r, self.cy / r, w, h)

    def as_floats(self) -> np.ndarray:
        """16 float64 values: R (row-major 9), t (3), fx, fy, cx, cy."""
        return np.concatenate([self.R.reshape(9), self.t,
                               [self.fx, self.fy, self.cx, self.cy]]).astype(np.float64)


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int
    cameras: list
    targets: list            # per camera: float32 [3][H][W]
    bg: np.ndarray           # (3,) float32

    @property
    def n(self) -> int:
        return int(self.means.shape[1])


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """World->camera (R, t) for a camera at `eye` looking at `target`, OpenCV axes."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ eye
    return R, t


def ring_camera(angle, radius, width, height, fov_x_deg=60.0, height_z=0.0):
    R, t = look_at((radius * math.cos(angle), radius * math.sin(angle), height_z))
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(R, t, fx, fx, width / 2.0, height / 2.0, width, height)


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    return q / np.linalg.norm(q, axis=0, keepdims=True)


def _sh_coeffs(rng, n, deg, dc_lo, dc_hi, rest_sigma):
    k = (deg + 1) ** 2
    sh = np.empty((k, 3, n), np.float64)
    sh[0] = rng.uniform(dc_lo, dc_hi, (3, n))
    if k > 1:
        sh[1:] = rng.normal(0.0, rest_sigma, (k - 1, 3, n))
    return sh


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32))


def tiny_scene(seed=0, n=2000, width=128, height=128, sh_degree=0):
    """Plain single view: 2,000 Gaussians, 128x128, SH degree 0.

    means U([-1,1]^2 x [2,6]); log-scales N(-3, 0.5^2); quaternions N(0, I4)
    normalised; logits N(0,1); rgb U(0,1); identity pose, fx=fy=128, cx=cy=64;
    target U(0,1); black background.
    """
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)])
    log_scales = rng.normal(-3.0, 0.5, (3, n))
    quats = _unit_quats(rng, n)
    logits = rng.normal(0.0, 1.0, n)
    sh = _sh_coeffs(rng, n, sh_degree, -_DC_HALF_RANGE_FOR_UNIT_RGB,
                    _DC_HALF_RANGE_FOR_UNIT_RGB, 0.05)
    cam = Camera(np.eye(3), np.zeros(3), 128.0 * width / 128, 128.0 * height / 128,
                 width / 2.0, height / 2.0, width, height)
    target = rng.uniform(0, 1, (3, height, width))
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh),
                 sh_degree, [cam], [_f32(target)], np.zeros(3, np.float32))


def box_scene(seed=1, n=1_000_000, cams=None, sh_degree=3, box=5.0,
              log_scale_mu=-4.0, log_scale_sigma=0.7, logit_mu=0.0, logit_sigma=1.0,
              with_targets=True):
    """Gaussians uniform in a 10-unit box around a camera ring (radius 4, z = 0).

    log-scales N(-4, 0.7^2); quaternions N(0, I4); logits N(0,1);
    SH degree 3 with DC U(0,1) and the rest N(0, 0.05^2); target U(0,1).
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(-box, box, (3, n))
    log_scales = rng.normal(log_scale_mu, log_scale_sigma, (3, n))
    quats = rng.standard_normal((4, n))
    logits = rng.normal(logit_mu, logit_sigma, n)
    sh = _sh_coeffs(rng, n, sh_degree, 0.0, 1.0, 0.05)
    if cams is None:
        cams = [ring_camera(0.0, 4.0, 1600, 1040)]
    targets = []
    if with_targets:
        for c in cams:
            targets.append(_f32(rng.uniform(0, 1, (3, c.height, c.width))))
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh),
                 sh_degree, cams, targets, np.zeros(3, np.float32))


def single_view_1m(seed=1, n=1_000_000, with_targets=True):
    """One 1600x1040 view of 1,000,000 Gaussians, SH degree 3 (fwd+bwd+stats)."""
    return box_scene(seed=seed, n=n, with_targets=with_targets)


# Coarse-to-fine resolution mix of the batched step: factors r per view.
BATCHED_FACTORS = (4, 4, 2, 2, 2, 1, 1, 1)


def batched_c2f(seed=2, n=500_000, with_targets=True, factors=BATCHED_FACTORS):
    """Eight views on the radius-4 ring at mixed resolutions (2x400x260,
    3x800x520, 3x1600x1040), 500,000 Gaussians, SH degree 3."""
    rng = np.random.default_rng(seed + 1000)
    angles = rng.uniform(0, 2 * math.pi, len(factors))
    cams = [ring_camera(a, 4.0, 1600, 1040).scaled(r) for a, r in zip(angles, factors)]
    return box_scene(seed=seed, n=n, cams=cams, with_targets=with_targets)


@dataclasses.dataclass
class DensifyInputs:
    log_scales: np.ndarray       # [3][N]
    quats: np.ndarray            # [4][N]
    means: np.ndarray            # [3][N]
    opacity_logits: np.ndarray   # [N]
    dmean2d: np.ndarray          # [V][2][N] pixel-space position gradients
    visible: np.ndarray          # [V][N] int32 (1 = the Gaussian was rendered in that view)
    view_wh: np.ndarray          # [V][2] int32 image sizes (for the NDC scale)
    extent: float                # camera extent (1.1 x ring radius)


def densify_workload(seed=3, n=3_000_000, n_views=100, width=1600, height=1040):
    """Synthetic densification statistics over 100 views.

    Visibility ~ Bernoulli(0.5); per-Gaussian gradient magnitude
    m_i = 2e-4 * exp(N(-1.5, 1)) / sqrt(pi/2); per-view NDC gradient m_i * N(0, I2)
    expressed in pixel units (divided by (W/2, H/2)).  logits N(-2, 1.5^2),
    other parameters as in the box scene.  Camera extent 1.1 * 4.
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(-5, 5, (3, n))
    log_scales = rng.normal(-4.0, 0.7, (3, n))
    quats = rng.standard_normal((4, n))
    logits = rng.normal(-2.0, 1.5, n)
    mag = 2e-4 * np.exp(rng.normal(-1.5, 1.0, n)) / math.sqrt(math.pi / 2)
    vis = np.empty((n_views, n), np.int32)
    g = np.empty((n_views, 2, n), np.float32)
    for v in range(n_views):
        vis[v] = rng.random(n) < 0.5
        z = rng.standard_normal((2, n))
        g[v, 0] = mag * z[0] / (width / 2.0)
        g[v, 1] = mag * z[1] / (height / 2.0)
    wh = np.tile(np.array([[width, height]], np.int32), (n_views, 1))
    return DensifyInputs(_f32(log_scales), _f32(quats), _f32(means), _f32(logits),
                         g, vis, wh, 1.1 * 4.0)


def procedural_scene(seed=4, n=6_000_000, n_spheres=64, n_planes=16, sh_degree=3):
    """Gaussians sampled on random spheres and planes (a structured scene).

    64 spheres (radius U(0.2, 1)) and 16 planes (2x2) in [-4, 4]^3, surfels flat
    along the surface normal (log-scale N(-6, 0.3^2) along it, N(-4.5, 0.3^2) in
    the tangent plane), logits N(1, 1), per-primitive DC colour, higher SH
    N(0, 0.05^2).
    """
    rng = np.random.default_rng(seed)
    n_prims = n_spheres + n_planes
    prim = rng.integers(0, n_prims, n)
    centres = rng.uniform(-4, 4, (n_prims, 3))
    radii = rng.uniform(0.2, 1.0, n_spheres)
    normals_pl = rng.standard_normal((n_planes, 3))
    normals_pl /= np.linalg.norm(normals_pl, axis=1, keepdims=True)
    colours = rng.uniform(0, 1, (n_prims, 3))
    means = np.empty((n, 3))
    normals = np.empty((n, 3))
    sph = prim < n_spheres
    d = rng.standard_normal((int(sph.sum()), 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    means[sph] = centres[prim[sph]] + radii[prim[sph], None] * d
    normals[sph] = d
    pl = ~sph
    k = prim[pl] - n_spheres
    nrm = normals_pl[k]
    a = np.cross(nrm, np.array([0.0, 0.0, 1.0]))
    bad = np.linalg.norm(a, axis=1) < 1e-6
    a[bad] = np.cross(nrm[bad], np.array([1.0, 0.0, 0.0]))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.cross(nrm, a)
    uv = rng.uniform(-1, 1, (int(pl.sum()), 2))
    means[pl] = centres[prim[pl]] + uv[:, :1] * a + uv[:, 1:] * b
    normals[pl] = nrm
    # Rotation taking the local z axis to the normal: quaternion from z to n.
    z = np.array([0.0, 0.0, 1.0])
    w = 1.0 + normals @ z
    xyz = np.cross(np.broadcast_to(z, normals.shape), normals)
    q = np.concatenate([w[:, None], xyz], axis=1)
    flip = w < 1e-6
    q[flip] = np.array([0.0, 1.0, 0.0, 0.0])
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    log_scales = np.empty((3, n))
    log_scales[0] = rng.normal(-4.5, 0.3, n)
    log_scales[1] = rng.normal(-4.5, 0.3, n)
    log_scales[2] = rng.normal(-6.0, 0.3, n)
    logits = rng.normal(1.0, 1.0, n)
    kk = (sh_degree + 1) ** 2
    sh = np.empty((kk, 3, n))
    sh[0] = ((colours[prim] - 0.5) * 2.0 * _DC_HALF_RANGE_FOR_UNIT_RGB).T
    if kk > 1:
        sh[1:] = rng.normal(0.0, 0.05, (kk - 1, 3, n))
    return Scene(_f32(means.T), _f32(log_scales), _f32(q.T), _f32(logits), _f32(sh),
                 sh_degree, [], [], np.zeros(3, np.float32))


def procedural_cameras(seed=4, n_cams=64, radius=6.0, width=1920, height=1080):
    rng = np.random.default_rng(seed + 2000)
    angles = rng.uniform(0, 2 * math.pi, n_cams)
    heights = rng.uniform(-1.0, 1.0, n_cams)
    return [ring_camera(a, radius, width, height, height_z=h) for a, h in zip(angles, heights)]


def random_scene(seed, n, width, height, sh_degree=3, depth=(1.5, 5.0), spread=1.0,
                 log_scale=(-3.0, 0.5), logit=(0.0, 1.0), n_views=1):
    """Small scenes for exhaustive parity: Gaussians in front of a camera at the
    origin (or on a small ring of views), sized so every tile and a ragged edge
    tile are exercised."""
    rng = np.random.default_rng(seed)
    aspect = width / height
    means = np.stack([rng.uniform(-spread * aspect, spread * aspect, n) * 0.6,
                      rng.uniform(-spread, spread, n) * 0.6,
                      rng.uniform(depth[0], depth[1], n)])
    log_scales = rng.normal(log_scale[0], log_scale[1], (3, n))
    quats = rng.standard_normal((4, n))
    logits = rng.normal(logit[0], logit[1], n)
    sh = _sh_coeffs(rng, n, sh_degree, 0.0, 1.0, 0.1)
    f = 0.8 * width
    cams = []
    for v in range(n_views):
        ang = 0.15 * v
        R, _ = look_at((0.0, 0.0, 0.0), (math.sin(ang), 0.0, math.cos(ang)), up=(0.0, -1.0, 0.0))
        cams.append(Camera(R, np.zeros(3), f, f, width / 2.0 + 0.3, height / 2.0 - 0.2,
                           width, height))
    targets = [_f32(rng.uniform(0, 1, (3, c.height, c.width))) for c in cams]
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh),
                 sh_degree, cams, targets, np.zeros(3, np.float32))
