"""Training driver of the paper's method on one GPU, built from the library's
calls: per iteration the coarse-to-fine schedule picks the resolution, one
view is rendered and differentiated (projection, binning, compositing, loss of
Eq. 3, compositing adjoint, projection adjoint with the densification
statistic), and sparse Adam updates the rendered Gaussians; inside the
densification window, every `interval` iterations the global-to-local policy
selects split and clone candidates (clones suppressed in the global phase),
the adaptive opacity threshold selects the pruned ones, and the compaction
rebuilds parameters and optimiser state; opacities are reset periodically
(Methodology; Preliminary; Experiments, implementation details).  With
lineage=True every Gaussian also carries the attributes of the Spatial
diffusion analysis (its parent point's original position and the splits and
clones on its line of descent), carried through each compaction;
footprint_3sigma=True bins by the original 3DGS 3-sigma squares.

Every numerical step runs in libgsmi.so; this module keeps the tensors and
the iteration logic.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gsmi, schedule

PARAMS = gsmi.PARAM_NAMES                       # means, log_scales, quats, opacity_logits, sh
ROWS_POLICY = {"means": gsmi.ATTR_MEAN, "log_scales": gsmi.ATTR_LOGSCALE, "quats": gsmi.ATTR_COPY,
               "opacity_logits": gsmi.ATTR_COPY, "sh": gsmi.ATTR_COPY}
LINEAGE_POLICY = {"origin": gsmi.ATTR_COPY, "splits": gsmi.ATTR_SPLIT_COUNT,
                  "clones": gsmi.ATTR_CLONE_COUNT}


class Trainer:
    def __init__(self, params: dict, sh_degree: int, cameras, targets, policy, extent: float,
                 lrs=None, lam: float = 0.2, seed: int = 0, device="cuda", capacity=None,
                 lineage: bool = False, footprint_3sigma: bool = False,
                 spatial_order: bool = True):
        self.dev = torch.device(device)
        self.p = {k: params[k].to(self.dev).contiguous().clone() for k in PARAMS}
        self.sh_degree = sh_degree
        self.cameras = list(cameras)
        self.targets = [torch.as_tensor(t, dtype=torch.float32).to(self.dev) for t in targets]
        self.policy = policy
        self.extent = extent
        self.lam = lam
        self.lrs = dict(log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh=2.5e-3)
        if lrs:
            self.lrs.update(lrs)
        self.rng = np.random.default_rng(seed)
        self.seed = seed
        self.capacity = capacity
        # sparse Adam reads the gradient rows of rendered Gaussians only
        self.opts = gsmi.raster_opts(footprint_3sigma=footprint_3sigma, grad_rendered_only=True)
        # keep the Gaussians in spatial (Morton) order after every densification:
        # the projection, its adjoint and sparse Adam then skip whole waves of
        # Gaussians the view does not render
        self.spatial_order = spatial_order
        self._reset_state()
        # original position [3][n], split count [1][n], clone count [1][n] (FP32)
        self.lineage = None
        if lineage:
            self.lineage = {"origin": self.p["means"].clone(),
                            "splits": torch.zeros(1, self.n, device=self.dev),
                            "clones": torch.zeros(1, self.n, device=self.dev)}
        self._frames = {}
        self._targets = {}
        self.history = []          # (iteration, loss, n, resolution)
        self.densify_log = []      # (iteration, n_in, n_out, clones, splits, pruned, mode)

    @property
    def n(self) -> int:
        return int(self.p["means"].shape[-1])

    def _reset_state(self):
        self.m = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.accum = torch.zeros(self.n, device=self.dev)
        self.denom = torch.zeros(self.n, device=self.dev)
        self.t = 0

    def _frame(self, cam):
        key = (self.n, cam.width, cam.height)
        f = self._frames.get(key)
        if f is None:
            cap = self.capacity or max(1 << 20, 64 * ((cam.width + 15) // 16) * ((cam.height + 15) // 16))
            f = gsmi.Frame(self.n, [(cam.width, cam.height)], cap, self.dev)
            self._frames = {k: v for k, v in self._frames.items() if k[0] == self.n}
            self._frames[key] = f
        return f

    def _target(self, view: int, r: int):
        key = (view, r)
        t = self._targets.get(key)
        if t is None:
            t = schedule.downscale(self.targets[view], r).contiguous()
            self._targets[key] = t
        return t

    def step(self, it: int) -> float:
        r = self.policy.schedule.resolution(it)
        view = int(self.rng.integers(len(self.cameras)))
        cam = self.cameras[view].scaled(r)
        target = self._target(view, r)
        frame = self._frame(cam)
        cams_dev = gsmi.cameras_to_device([cam], self.dev)
        while True:
            frame.project(self.p, self.sh_degree, cams_dev, self.opts)
            image = frame.render(self.opts)
            nv, ni, ovf = frame.status(raise_on_overflow=False)
            if not ovf:
                break
            self._frames.pop((self.n, cam.width, cam.height), None)
            self.capacity = max(2 * frame.cap, ni)
            frame = self._frame(cam)
        loss, dL = gsmi.ssim_loss_grad(image.view(3, cam.height, cam.width), target, self.lam)
        frame.render_backward(self.opts, dL.reshape(-1))
        self.t += 1
        lrs = dict(self.lrs, means=self.policy.position_lr(it, self.extent))
        # sparse Adam inside the projection adjoint: each Gaussian's summed
        # gradients go from registers into the update, none reaches memory
        adam = gsmi.FusedAdamStep({k: (self.m[k], self.v[k]) for k in PARAMS}, lrs, self.t)
        frame.project_backward(self.p, self.sh_degree, cams_dev, self.opts, {}, self.accum,
                               self.denom, adam=adam)
        value = float(loss)
        self.history.append((it, value, self.n, r))
        if self.policy.densify_now(it):
            self.densify(it)
        if self.policy.opacity_reset_now(it):
            self.reset_opacity()
        return value

    def densify(self, it: int):
        g, ls_thr, lo_upper = self.policy.thresholds(self.extent)
        mode = self.policy.densify_mode(it)
        # adaptive opacity threshold tau = min(alpha_sorted[floor(N p)], tau_u), in logit space
        thr, _ = gsmi.adaptive_prune_threshold(self.p["opacity_logits"], p=self.policy.prune_ratio,
                                               tau_u=self.policy.prune_upper)
        split, clone, prune = gsmi.densify_select(self.accum, self.denom, self.p["log_scales"],
                                                  self.p["opacity_logits"], g, ls_thr,
                                                  float(thr.item()), mode)
        src, kind, n_out = gsmi.densify_plan(split, clone, prune)
        n_in = self.n
        if n_out == 0:
            return
        attrs, names = [], []
        for k in PARAMS:
            rows = self.p[k].numel() // n_in
            attrs.append((self.p[k].reshape(rows, n_in), rows, ROWS_POLICY[k]))
            names.append(("p", k))
            for st in ("m", "v"):
                attrs.append((getattr(self, st)[k].reshape(rows, n_in), rows, gsmi.ATTR_ZERO_NEW))
                names.append((st, k))
        if self.lineage is not None:
            for k, policy in LINEAGE_POLICY.items():
                a = self.lineage[k]
                attrs.append((a, a.shape[0], policy))
                names.append(("lineage", k))
        outs = gsmi.densify_apply(src, kind, n_in, attrs, self.p["means"], self.p["log_scales"],
                                  self.p["quats"], self.seed, it)
        shapes = {k: self.p[k].shape[:-1] for k in PARAMS}
        for (st, k), o in zip(names, outs):
            if st == "lineage":
                self.lineage[k] = o.contiguous()
            else:
                getattr(self, st)[k] = o.reshape(*shapes[k], n_out).contiguous()
        if self.spatial_order:
            osrc, okind = gsmi.spatial_order(self.p["means"])
            keys = [(st, k) for st in ("p", "m", "v") for k in PARAMS]
            tensors = [getattr(self, st)[k] for st, k in keys]
            if self.lineage is not None:
                keys += [("lineage", k) for k in LINEAGE_POLICY]
                tensors += [self.lineage[k] for k in LINEAGE_POLICY]
            for (st, k), o in zip(keys, gsmi.reorder(tensors, osrc, okind)):
                (self.lineage if st == "lineage" else getattr(self, st))[k] = o.contiguous()
        self.accum = torch.zeros(n_out, device=self.dev)
        self.denom = torch.zeros(n_out, device=self.dev)
        kinds = torch.bincount(kind.to(torch.int64), minlength=4).tolist()
        self.densify_log.append((it, n_in, n_out, kinds[gsmi.KIND_CLONE], kinds[gsmi.KIND_SPLIT0],
                                 int(prune.sum()), mode))

    def reset_opacity(self, ceiling: float = 0.01):
        """Opacities above the ceiling are set to it (logit space); their
        moments restart from zero."""
        lim = math.log(ceiling / (1.0 - ceiling))
        self.p["opacity_logits"].clamp_(max=lim)
        self.m["opacity_logits"].zero_()
        self.v["opacity_logits"].zero_()

    def lineage_summary(self):
        """Per category of the Spatial diffusion analysis -- split-dominated
        (more splits than clones on the line of descent), clone-dominated, equal
        -- the number of Gaussians and their mean distance from the original
        position of their parent point.  Host-side analysis of the lineage
        attributes (requires lineage=True)."""
        if self.lineage is None:
            raise RuntimeError("the trainer was built without lineage=True")
        s = self.lineage["splits"][0].cpu().numpy()
        c = self.lineage["clones"][0].cpu().numpy()
        d = np.linalg.norm((self.p["means"] - self.lineage["origin"]).cpu().numpy().astype(np.float64),
                           axis=0)
        out = {}
        for name, sel in (("split", s > c), ("clone", c > s), ("equal", s == c)):
            out[name] = (int(sel.sum()), float(d[sel].mean()) if sel.any() else float("nan"))
        return out
