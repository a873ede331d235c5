"""Autotuner for the rasterizer launch shape.

Searches the LDS batch size (splats staged per batch: 64, 128, 256), the
work distribution (one workgroup per (view, tile) with one wave and a 2x2
quad per lane or four waves and one pixel per lane, or a persistent grid of
2048 / 4096 / 8192 single waves pulling tiles heaviest-first from a queue),
how the per-tile lists are put in depth order (a sort per tile, or a depth
presort of the visible entries) and the digit split of the radix sort by tile
(60 candidates), by timing the captured training step of the given views, and
caches the winner per (device, workload signature) in a JSON file
($GSMI_AUTOTUNE_CACHE, default ~/.cache/gsmi_autotune.json).
"""
from __future__ import annotations

import json
import os

import torch

from . import gsmi

BATCHES = (64, 128, 256)
PERSISTENT = (0, 2048, 4096, 8192)
# how each tile's list gets its depth order: per-tile sorts, or a depth presort of
# the visible entries (long lists favour the presort); and the digit split of the
# radix sort by tile (8-bit digits, or digits of equal width)
PRESORT = (False, True)
BALANCED = (False, True)
# lanes of the compositing kernels on the plain grid: one pixel (four waves per
# tile) or a 2x2 quad (one wave per tile); persistent grids take quads
LANES = ("pixels", "quads")
SHAPE_KEYS = ("raster_batch", "persistent_blocks", "depth_presort", "balanced_digits", "lanes")


def n_candidates():
    per_sort = len(PRESORT) * len(BALANCED)
    return len(BATCHES) * per_sort * (len(LANES) + len(PERSISTENT) - 1)


def opts_of(best, **other):
    """gsmi.raster_opts for a tuned shape (the other options as given)."""
    return gsmi.raster_opts(**{k: best[k] for k in SHAPE_KEYS if k in best}, **other)


def _cache_path():
    return os.environ.get("GSMI_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gsmi_autotune.json"))


def _signature(n, cams, sh_degree, opts=None):
    dev = torch.cuda.get_device_name(0)
    sizes = ",".join("%dx%d" % (c.width, c.height) for c in cams)
    extra = ""
    if opts and opts.get("footprint_3sigma"):
        extra = "|3sigma"
    # the candidate set is part of the signature: a cache written for another set
    # is not reused
    return "%s|n=%d|sh=%d|%s%s|%d candidates" % (dev, n, sh_degree, sizes, extra, n_candidates())


def _load():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _time_step(frame, params, sh_degree, cams_dev, opts, images, targets, scale, loss, dL, grads,
               reps=5):
    g = gsmi.StepGraph(frame, params, sh_degree, cams_dev, opts, images, targets, scale, loss, dL,
                       grads)
    for _ in range(2):
        g.launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.launch()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_batched(scene, cams, params, device, cap=32 << 20, use_cache=True, opts=None):
    """Best {raster_batch, persistent_blocks, ms} for a step over `cams`.
    opts: the other gsmi.raster_opts arguments (background, near plane,
    footprint), kept fixed."""
    opts = dict(opts or {})
    sig = _signature(scene.n, cams, scene.sh_degree, opts)
    cache = _load() if use_cache else {}
    if sig in cache:
        return cache[sig]
    frame = gsmi.Frame(scene.n, [(c.width, c.height) for c in cams], cap, device)
    cams_dev = gsmi.cameras_to_device(cams, device)
    images = torch.empty(frame.image_numel(), device=device)
    targets = torch.rand(frame.image_numel(), device=device)
    loss = torch.zeros(1, device=device)
    dL = torch.empty_like(images)
    grads = gsmi.empty_grads(params)
    scale = 1.0 / images.numel()
    results = []
    for b in BATCHES:
        for pb in PERSISTENT:
            for ps in PRESORT:
                for bd in BALANCED:
                    for ln in (LANES if pb == 0 else ("quads",)):
                        shape = {"raster_batch": b, "persistent_blocks": pb, "depth_presort": ps,
                                 "balanced_digits": bd, "lanes": ln}
                        o = opts_of(shape, **opts)
                        ms = _time_step(frame, params, scene.sh_degree, cams_dev, o, images,
                                        targets, scale, loss, dL, grads)
                        results.append(dict(shape, ms=round(ms, 4)))
    best = dict(min(results, key=lambda r: r["ms"]))
    best["candidates"] = len(results)
    cache[sig] = best
    if use_cache:
        _store(cache)
    return best
