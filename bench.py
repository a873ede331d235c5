#!/usr/bin/env python3
"""Benchmark of the Gaussian-splatting hot path on one MI355X (gfx950).

Metric: milliseconds per training iteration's forward + backward at
1,000,000 Gaussians, one 1600x1040 view, SH degree 3, FP32: projection ->
tile binning (prefix sums + radix sorts) -> front-to-back compositing -> L1
loss and its gradient -> compositing adjoint -> chain rule to the raw
parameters with the densification statistic fused.  All inputs are resident
in HBM before the timed region; the step is timed both as a captured hipGraph
and as eager launches, K steps between two synchronisations, and the faster
of the two is the value.

Also reported, each on its own synthetic workload:
  - the plain 128x128 step (2,000 Gaussians, SH0);
  - the batched coarse-to-fine step (8 views at 400x260, 800x520 and
    1600x1040 in one frame, 500,000 Gaussians) against the same 8 views
    stepped one at a time;
  - the roofline position of the dominant kernel (the compositing adjoint,
    timed live with HIP events on the stream it runs on) and, for every
    HBM-bound stage, its algorithmic bytes over its live time;
  - Eq. 3's loss with D-SSIM, sparse Adam, and one densification of
    3,000,000 Gaussians (median of 20 calls each);
  - 200 training steps at 6,000,000 Gaussians and four 1920x1080 views per
    step through the torch.autograd.Function (Eq. 3 loss against renders of
    the unperturbed scene, sparse Adam), mean ms over steps 11-200;
  - the FP64 CPU oracle on this host's cores, on all of them and on one,
    for each of those workloads (bounded samples where a full run would take
    hours; each sample is described in the output).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batched]
                       [--no-extras] [--c5-steps 200]
"""
import argparse
import hashlib
import json
import math
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles at 2.4 GHz
VALU_ISSUE_PEAK_G = 256 * 4 * 2.4 / 4
# FP32 vector peak: 256 CUs x 128 FP32 lanes (packed / dual issue) x 2 flop (FMA) x 2.4 GHz;
# without packed FP32 instructions (this library is built without them) half of that
FP32_PEAK_TFLOPS = 157.3
FP32_PEAK_NONPACKED_TFLOPS = 78.6
# The adjoint's arithmetic per (pixel, splat) pair walked: 60-80 VALU operations plus one
# exponential and one division re-evaluating alpha, transmittance and the nine partial
# derivatives; the midpoint is the model, counted as flop
BWD_FLOP_PER_PAIR = 70
# Algorithmic HBM bytes of the stages bound by memory (per unit of work):
#   projection    12 B per Gaussian (means) + 276 B per visible Gaussian (the other
#                 parameters read, the projected splat written)
#   binning       8 B per Gaussian (counts and their scan) + 44 B per tile instance (emission,
#                 one read and one write of each key-value pair, tile ranges)
#   chain rule    524 B per visible Gaussian-view (parameters and splat gradients read,
#                 parameter gradients and the statistic written)
#   statistic     12 B per Gaussian-view (rendered flag and position gradient read) + 16 B per
#                 Gaussian (the two accumulators read and written once: the kernel keeps
#                 them in registers across the views of a launch)
#   selection     27 B per Gaussian (statistic and scales read, three masks written)
#   densify       3 B per parent (masks) + 5 B per output row (map), and 708 B per surviving
#                 parent read and per output row written (parameters and two Adam moments)
#   sparse Adam   28 B per parameter float of every rendered Gaussian (parameter, gradient and
#                 two moments read, parameter and moments written) + 4 B per Gaussian-view
#                 (the rendered flag)
PROJ_B_PER_G, PROJ_B_PER_VIS = 12, 276
BIN_B_PER_G, BIN_B_PER_INST = 8, 44
CHAIN_B_PER_VIS = 524
STATS_B_PER_GV, STATS_B_PER_G = 12, 16
SELECT_B_PER_G = 27
ADAM_B_PER_FLOAT = 28
PARAM_FLOATS = 59          # floats per Gaussian at SH degree 3
PARAM_BYTES = 4 * PARAM_FLOATS


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--profile", action="store_true",
                    help="minimal run for a profiler: metric workload only, no CPU leg")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the loss, Adam, densification and 6M training timings")
    ap.add_argument("--c5-steps", type=int, default=200,
                    help="training steps of the 6M-Gaussian workload (timed: steps 11..)")
    ap.add_argument("--profile-workload",
                    choices=("batched_8_views", "step_6m_4_views", "plain_128x128"),
                    help="for a profiler: time only this workload with the launch shape given by "
                         "--raster-batch / --persistent / --presort / --balanced / --lanes and "
                         "print one JSON line")
    ap.add_argument("--raster-batch", type=int, default=0)
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--presort", action="store_true")
    ap.add_argument("--balanced", action="store_true")
    ap.add_argument("--lanes", choices=("pixels", "quads"), default=None,
                    help="lane layout of the compositing kernels (default: by frame size)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def to_dev(sc, dev, torch, gsmi):
    return {k: torch.from_numpy(getattr(sc, k)).to(dev).contiguous() for k in gsmi.PARAM_NAMES}


# composite_l1: compositing with the L1 term of Eq. 3 fused into its pixel writes
STAGES = ["project", "bin", "composite_l1", "render_backward", "project_backward"]


class Step:
    """One training step's buffers and its captured graph for a set of views."""

    def __init__(self, sc, cams, params, opts, cap, torch, gsmi, dev):
        self.torch, self.gsmi = torch, gsmi
        self.sc, self.cams, self.params, self.opts = sc, cams, params, opts
        self.frame = gsmi.Frame(sc.n, [(c.width, c.height) for c in cams], cap, dev)
        self.cams_dev = gsmi.cameras_to_device(cams, dev)
        self.images = torch.empty(self.frame.image_numel(), device=dev)
        if sc.targets:
            self.targets = torch.cat([torch.from_numpy(t).reshape(-1) for t in sc.targets]).to(dev)
        else:
            self.targets = torch.rand(self.frame.image_numel(), device=dev)
        self.loss = torch.zeros(1, device=dev)
        self.dL = torch.empty_like(self.images)
        self.grads = gsmi.empty_grads(params)
        self.acc = torch.zeros(sc.n, device=dev)
        self.den = torch.zeros(sc.n, device=dev)
        self.l1_scale = 1.0 / self.images.numel()
        self.graph = None

    def eager(self, events=None):
        f, g = self.frame, self.gsmi
        ev = events
        if ev: ev[0].record()
        f.project(self.params, self.sc.sh_degree, self.cams_dev, self.opts)
        if ev: ev[1].record()
        f.bin(self.opts)
        if ev: ev[2].record()
        self.loss.zero_()
        f.composite_l1(self.opts, self.images, self.targets, self.l1_scale, self.loss, self.dL)
        if ev: ev[3].record()
        f.render_backward(self.opts, self.dL)
        if ev: ev[4].record()
        f.project_backward(self.params, self.sc.sh_degree, self.cams_dev, self.opts, self.grads,
                           self.acc, self.den)
        if ev: ev[5].record()

    def capture(self):
        self.graph = self.gsmi.StepGraph(self.frame, self.params, self.sc.sh_degree, self.cams_dev,
                                         self.opts, self.images, self.targets, self.l1_scale,
                                         self.loss, self.dL, self.grads, self.acc, self.den)

    def launch(self):
        self.graph.launch()

    def checked(self):
        """Visible entries and instances of the last render; raises if the
        instance capacity overflowed (the step would then time less work)."""
        nv, ni, _ = self.frame.status()
        return nv, ni


def time_loop(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def paired_loops(torch, fa, fb, steps, warmup, rounds=4):
    """Two launch forms of one step timed in alternating blocks of `steps`
    steps (a b b a a b b a ...), each block bracketed by synchronisations, so
    neither takes the clock ramp or drift of its position; the median block of
    each."""
    for _ in range(warmup):
        fa()
        fb()
    ta, tb = [], []
    for r in range(rounds):
        for which in ((0, 1) if r % 2 == 0 else (1, 0)):
            (ta if which == 0 else tb).append(time_loop(torch, (fa, fb)[which], steps, 0))
    return statistics.median(ta), statistics.median(tb)


def median_events(torch, fn, reps, setup=None):
    """Median over reps of fn's duration between two events on the current
    stream (setup, if given, runs before each rep outside the timed pair)."""
    out = []
    for _ in range(reps):
        if setup:
            setup()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return statistics.median(out)


def breakdown(torch, step, reps):
    """Median per-stage time of eager steps, events between the stage calls."""
    acc = [[] for _ in STAGES]
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(STAGES) + 1)]
        step.eager(ev)
        torch.cuda.synchronize()
        for i in range(len(STAGES)):
            acc[i].append(ev[i].elapsed_time(ev[i + 1]))
    return {n: statistics.median(a) for n, a in zip(STAGES, acc)}


def hbm_line(stage, workload, nbytes, ms):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"stage": stage, "workload": workload, "algorithmic_bytes": int(nbytes),
            "ms": round(ms, 4), "achieved_gbs": round(gbs, 1), "peak_gbs": HBM_PEAK_GBS,
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def source_hash(*files):
    """Hash of the code of the given sources, comments and blank space aside,
    so a counter summary stays valid across comment edits."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def counter_values(kernel_src_hash):
    """Per-launch counter values of the adjoint kernel from the committed
    rocprofv3 summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "raster_bwd_1m_1600x1040_counters.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    for ln in open(path):
        if "=" in ln and not ln.startswith("#"):
            k, v = ln.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_src_hash:
        return {}
    out = {}
    for k in ("hbm_bytes_per_launch", "valu_instructions"):
        try:
            out[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    return out


def timed(torch, fn, steps, warmup):
    return time_loop(torch, fn, steps, warmup)


# ---------------------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------------------
def metric_leg(torch, gsmi, sc, params, dev, K, W, label, rendered_only=False):
    """The 1M-Gaussian 1600x1040 step: graph and eager timing, per-stage
    breakdown, the adjoint's roofline, and the HBM-bound stages' algorithmic
    bytes over their live times.  rendered_only: the projection adjoint writes
    the gradient rows of rendered Gaussians only (what sparse Adam reads)."""
    opts = gsmi.raster_opts(grad_rendered_only=rendered_only)
    st = Step(sc, sc.cameras, params, opts, 16 << 20, torch, gsmi, dev)
    st.eager()
    nvis, ninst = st.checked()
    log("%s: visible %d instances %d" % (label, nvis, ninst))
    st.capture()
    ms_graph, ms_eager = paired_loops(torch, st.launch, st.eager, K, W)
    st.checked()
    log("%s: 1M-Gaussian 1600x1040 step: graph %.3f ms eager %.3f ms" % (label, ms_graph, ms_eager))
    parts = breakdown(torch, st, max(5, K))
    log("%s: breakdown %s" % (label, json.dumps({k: round(v, 4) for k, v in parts.items()})))

    # dominant kernel: the compositing adjoint (one kernel per gs_render_backward call)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    # the renders before each timed adjoint also count the composited splats
    copts = gsmi.raster_opts(count_composited=True)
    for i in range(K):
        st.frame.project(params, sc.sh_degree, st.cams_dev, opts)
        st.frame.render(copts, st.images)
        ev[i][0].record()
        st.frame.render_backward(opts, st.dL)
        ev[i][1].record()
    torch.cuda.synchronize()
    bwd_ms = statistics.median(a.elapsed_time(b) for a, b in ev)
    n_contrib = st.frame.buffer(gsmi.BUF_N_CONTRIB).to(torch.int64).sum().item()
    n_comp = st.frame.buffer(gsmi.BUF_N_COMPOSITED).to(torch.int64).sum().item()
    flop = BWD_FLOP_PER_PAIR * n_contrib
    achieved = flop / (bwd_ms * 1e-3) / 1e12
    src_hash = source_hash("paper_2507_20239_amd/csrc/raster.hip",
                           "paper_2507_20239_amd/csrc/gs_internal.h")
    cv = counter_values(src_hash)
    valu = None
    if "valu_instructions" in cv:
        # wave64 VALU instructions per launch (SQ_INSTS_VALU) over the live launch time;
        # quarter-rate transcendentals count once but occupy four issue slots
        rate = cv["valu_instructions"] / (bwd_ms * 1e-3) / 1e9
        valu = {"wave_instructions": int(cv["valu_instructions"]), "achieved": round(rate, 1),
                "peak": VALU_ISSUE_PEAK_G, "unit": "G wave-instr/s",
                "frac": round(rate / VALU_ISSUE_PEAK_G, 4),
                "per_pair_walked": round(cv["valu_instructions"] * 64 / 4 / n_contrib, 2)}
    roofline = {"kernel": "raster_bwd_kernel (compositing adjoint)", "bound": "alu",
                "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": cv.get("hbm_bytes_per_launch"),
                "model": "%d flop per (pixel, splat) pair walked" % BWD_FLOP_PER_PAIR,
                "peak_nonpacked": FP32_PEAK_NONPACKED_TFLOPS,
                "frac_nonpacked": round(achieved / FP32_PEAK_NONPACKED_TFLOPS, 4),
                "launch_ms": round(bwd_ms, 4), "pairs_walked": int(n_contrib),
                "pairs_composited": int(n_comp), "valu_issue": valu, "source_hash": src_hash}
    wl = "1M Gaussians, 1600x1040, %d visible, %d instances, %s" % (nvis, ninst, label)
    hbm = [hbm_line("projection", wl, PROJ_B_PER_G * sc.n + PROJ_B_PER_VIS * nvis, parts["project"]),
           hbm_line("binning (scans, emission, radix sort, ranges, tile sort)", wl,
                    BIN_B_PER_G * sc.n + BIN_B_PER_INST * ninst, parts["bin"]),
           hbm_line("projection adjoint + statistic", wl, CHAIN_B_PER_VIS * nvis,
                    parts["project_backward"])]
    return {"ms": round(min(ms_graph, ms_eager), 4), "graph_ms": round(ms_graph, 4),
            "eager_ms": round(ms_eager, 4), "visible": nvis, "instances": ninst,
            "breakdown_ms": {k: round(v, 4) for k, v in parts.items()}, "roofline": roofline,
            "hbm": hbm}, st


def spatially_ordered(torch, gsmi, params, reps=5):
    """The Gaussians in spatial order, as the trainer keeps them: the
    permutation (gs_spatial_order) and its gather (gs_densify_apply) of the
    parameters and two optimiser moments of the same shapes; median times."""
    names = gsmi.PARAM_NAMES
    moments = [torch.zeros_like(params[k]) for k in names for _ in range(2)]
    t_order, t_gather = [], []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        src, kind = gsmi.spatial_order(params["means"])
        e[1].record()
        out = gsmi.reorder([params[k] for k in names] + moments, src, kind)
        e[2].record()
        torch.cuda.synchronize()
        t_order.append(e[0].elapsed_time(e[1]))
        t_gather.append(e[1].elapsed_time(e[2]))
    ordered = dict(zip(names, out[:len(names)]))
    return ordered, {"order_ms": round(statistics.median(t_order), 4),
                     "gather_params_and_moments_ms": round(statistics.median(t_gather), 4),
                     "note": "paid once per densification (every 100 iterations in 3DGS training), "
                             "not per step"}


def plain_128(torch, gsmi, synth, dev, K, W):
    """The plain single view: 2,000 Gaussians, 128x128, SH degree 0."""
    sc = synth.tiny_scene(seed=0)
    params = to_dev(sc, dev, torch, gsmi)
    st = Step(sc, sc.cameras, params, gsmi.raster_opts(), 1 << 20, torch, gsmi, dev)
    st.eager()
    nv, ni = st.checked()
    st.capture()
    reps = max(K, 100)
    g, e = paired_loops(torch, st.launch, st.eager, reps, W)
    return {"workload": "single view 128x128, 2,000 Gaussians, SH degree 0, fwd+bwd+statistic",
            "graph_ms": round(g, 4), "eager_ms": round(e, 4), "ms_per_step": round(min(g, e), 4),
            "visible": nv, "instances": ni, "steps": reps}, sc


def batched_leg(torch, gsmi, synth, dev, K, W):
    log("generating batched coarse-to-fine scene (500K, 8 views)")
    sb = synth.batched_c2f()
    # the Gaussians in the spatial order the trainer keeps (both forms use them)
    pb, _ = spatially_ordered(torch, gsmi, to_dev(sb, dev, torch, gsmi), reps=1)
    from paper_2507_20239_amd import autotune
    best = autotune.tune_batched(sb, sb.cameras, pb, dev, cap=32 << 20)
    bopts = autotune.opts_of(best)
    bst = Step(sb, sb.cameras, pb, bopts, 32 << 20, torch, gsmi, dev)
    bst.eager()
    nv, ni = bst.checked()
    bst.capture()
    ms_b, ms_b_eager = paired_loops(torch, bst.launch, bst.eager, K, W)
    bst.checked()
    plain = []
    popts = gsmi.raster_opts()
    counts = []
    for v, cam in enumerate(sb.cameras):
        one = synth.Scene(sb.means, sb.log_scales, sb.quats, sb.opacity_logits, sb.sh,
                          sb.sh_degree, [cam], [sb.targets[v]], sb.bg)
        s1 = Step(one, [cam], pb, popts, 16 << 20, torch, gsmi, dev)
        s1.eager()
        counts.append(s1.checked())
        s1.capture()
        plain.append(s1)

    def plain_graph():
        for s1 in plain:
            s1.launch()

    def plain_eager():
        for s1 in plain:
            s1.eager()

    ms_p, ms_p_eager = paired_loops(torch, plain_graph, plain_eager, K, W)
    for s1 in plain:
        s1.checked()
    best_plain = min(ms_p, ms_p_eager)
    best_batched = min(ms_b, ms_b_eager)
    log("batched %.3f ms (graph) %.3f ms (eager), plain %.3f ms (graph) %.3f ms (eager)"
        % (ms_b, ms_b_eager, ms_p, ms_p_eager))
    out = {"workload": "8 views (2x400x260, 3x800x520, 3x1600x1040), 500,000 Gaussians, SH3",
           "batched_graph_ms": round(ms_b, 4), "batched_eager_ms": round(ms_b_eager, 4),
           "plain_graph_ms": round(ms_p, 4), "plain_eager_ms": round(ms_p_eager, 4),
           "speedup": round(best_plain / best_batched, 3),
           "speedup_graph_vs_graph": round(ms_p / ms_b, 3),
           "visible_entries": nv, "instances": ni,
           "plain_instances": [c[1] for c in counts], "tuned": best}
    return out, sb


def extras(torch, gsmi, synth, st, params, sc, dev, reps=20):
    """Median-of-20 per-call times of the steps around the metric step: Eq. 3's
    loss with its D-SSIM term on the 1600x1040 image, the sparse Adam step over
    the 1M Gaussians (rendered ones updated), and one densification of the
    3,000,000-Gaussian workload (statistic over 100 views, selection, adaptive
    opacity threshold, compaction map, gather of parameters and Adam
    moments), each stage on fresh inputs."""
    out, hbm = {}, []
    img = st.images.view(3, 1040, 1600)
    tgt = st.targets.view(3, 1040, 1600)
    loss = torch.zeros(1, device=dev)
    grad = torch.empty_like(img)
    ws = torch.empty(3 * 4 * img.numel() + 4 * 3 * 6500, dtype=torch.uint8, device=dev)
    out["l1_dssim_loss_grad_ms"] = round(median_events(
        torch, lambda: gsmi.ssim_loss_grad(img, tgt, 0.2, loss, grad, ws), reps), 4)
    mom = {k: (torch.zeros_like(params[k]), torch.zeros_like(params[k])) for k in gsmi.PARAM_NAMES}
    pcopy = {k: params[k].clone() for k in gsmi.PARAM_NAMES}
    tt = st.frame.buffer(gsmi.BUF_TILES_TOUCHED)
    entries = [(pcopy[k], st.grads[k], mom[k][0], mom[k][1], 1e-3) for k in gsmi.PARAM_NAMES]
    cnt = [0]

    def adam():
        cnt[0] += 1
        gsmi.adam_step(entries, sc.n, cnt[0], tiles_touched=tt)

    adam_ms = median_events(torch, adam, reps)
    n_upd = int((tt > 0).sum().item())
    out["sparse_adam_ms"] = round(adam_ms, 4)
    out["rendered_gaussians"] = n_upd
    hbm.append(hbm_line("sparse Adam", "1M Gaussians, %d rendered" % n_upd,
                        ADAM_B_PER_FLOAT * PARAM_FLOATS * n_upd + 4 * sc.n, adam_ms))
    del mom, pcopy, entries

    log("generating the 3M-Gaussian densification workload (100 views)")
    d = synth.densify_workload()
    n = d.means.shape[1]
    V = int(d.dmean2d.shape[0])
    g = torch.from_numpy(d.dmean2d).to(dev)
    vis = torch.from_numpy(d.visible).to(dev)
    P = {"means": torch.from_numpy(d.means).to(dev), "log_scales": torch.from_numpy(d.log_scales).to(dev),
         "quats": torch.from_numpy(d.quats).to(dev),
         "opacity_logits": torch.from_numpy(d.opacity_logits).to(dev),
         "sh": torch.rand(48, n, device=dev)}
    acc = torch.zeros(n, device=dev)
    den = torch.zeros(n, device=dev)
    tg, tls, tlo = 2e-4, math.log(0.01 * d.extent), math.log(0.005 / 0.995)

    def fresh_stats():
        acc.zero_()
        den.zero_()

    t_stats = median_events(torch, lambda: gsmi.accumulate_densify_stats(g, vis, d.view_wh, acc, den),
                            reps, setup=fresh_stats)
    masks = {}

    def sel():
        masks["m"] = gsmi.densify_select(acc, den, P["log_scales"], P["opacity_logits"], tg, tls,
                                         tlo, True)

    t_sel = median_events(torch, sel, reps)
    t_thr = median_events(torch, lambda: gsmi.adaptive_prune_threshold(P["opacity_logits"], 0.03,
                                                                       0.05), reps)
    s_, c_, p_ = masks["m"]
    pruned = int(p_.sum().item())
    # the map without reading its length back (the timed call); then the length
    src = torch.empty(2 * n, dtype=torch.int32, device=dev)
    kind = torch.empty(2 * n, dtype=torch.uint8, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    t_plan = median_events(torch, lambda: gsmi.densify_plan_noalloc(s_, c_, p_, src, kind, n_out),
                           reps)
    m = int(n_out.item())
    src, kind = src[:m], kind[:m]
    pol = {"means": gsmi.ATTR_MEAN, "log_scales": gsmi.ATTR_LOGSCALE}
    attrs = []
    for k in gsmi.PARAM_NAMES:
        rows = P[k].numel() // n
        attrs.append((P[k].reshape(rows, n), rows, pol.get(k, gsmi.ATTR_COPY)))
        attrs.append((torch.zeros(rows, n, device=dev), rows, gsmi.ATTR_ZERO_NEW))
        attrs.append((torch.zeros(rows, n, device=dev), rows, gsmi.ATTR_ZERO_NEW))
    outs = gsmi.densify_apply(src, kind, n, attrs, P["means"], P["log_scales"], P["quats"], 0x5EED, 0)
    torch.cuda.synchronize()
    del outs

    def apply():
        gsmi.densify_apply(src, kind, n, attrs, P["means"], P["log_scales"], P["quats"], 0x5EED, 0)

    # each call allocates its 177 output rows from torch's cache (freed the call before)
    t_apply = median_events(torch, apply, reps)
    out["densify_3m"] = {
        "gaussians_in": n, "gaussians_out": m, "pruned": pruned, "views": V, "reps": reps,
        "stats_100_views_ms": round(t_stats, 4), "select_ms": round(t_sel, 4),
        "adaptive_threshold_ms": round(t_thr, 4), "plan_ms": round(t_plan, 4),
        "apply_params_and_moments_ms": round(t_apply, 4),
        "total_ms": round(t_stats + t_sel + t_thr + t_plan + t_apply, 4)}
    wl = "3M Gaussians, 100 views"
    hbm.append(hbm_line("densify statistic", wl, STATS_B_PER_GV * n * V + STATS_B_PER_G * n,
                        t_stats))
    hbm.append(hbm_line("densify select", wl, SELECT_B_PER_G * n, t_sel))
    a11 = 3 * n + 5 * m + 3 * PARAM_BYTES * (n - pruned) + 3 * PARAM_BYTES * m
    hbm.append(hbm_line("densify plan + apply (params and moments)", wl, a11, t_plan + t_apply))
    del P, g, vis, attrs
    torch.cuda.empty_cache()
    return out, hbm, d


def c5_training(torch, gsmi, synth, dev, steps, first_timed=11, warm=3):
    """The large training workload as configured: 6,000,000 Gaussians on
    spheres and planes, SH3, 64 ring cameras at 1920x1080, four random views
    per step through the torch.autograd.Function; targets are renders of the
    unperturbed scene, training starts from a perturbed copy (means +
    N(0, 0.01^2), DC + N(0, 0.1^2)); Eq. 3 loss (lambda 0.2), sparse Adam.
    Run twice from the same start and view sequence: eagerly, and as one
    captured graph of the whole step (rasterize, loss, backward, Adam)
    replayed from step warm + 1 on (the rasterizer checks its capacity
    lazily, takes its cameras from a device table, and Adam counts its steps
    on the device).  Returns mean ms over steps first_timed..steps and the
    first/last loss of each."""
    import numpy as np
    from paper_2507_20239_amd.autograd import GaussianRasterizer, photometric_loss
    log("generating the 6M-Gaussian procedural scene (64 cameras, 4 x 1920x1080 per step)")
    sc = synth.procedural_scene()
    cams = synth.procedural_cameras()
    names = gsmi.PARAM_NAMES
    P0 = {k: torch.from_numpy(np.ascontiguousarray(getattr(sc, k))).to(dev) for k in names}
    # the generator draws each Gaussian's primitive at random; the trainer keeps the
    # Gaussians in spatial order (gs_spatial_order at every densification)
    P0, reorder = spatially_ordered(torch, gsmi, P0, reps=1)
    r = GaussianRasterizer(sc.n, cams[:4], sc.sh_degree, device=dev, autotune=True,
                           lazy_overflow=True)
    table = gsmi.cameras_to_device(cams, dev).view(len(cams), -1)
    log("rendering the 64 target views")
    targets = torch.empty(len(cams), 3, 1080, 1920, device=dev)
    with torch.no_grad():
        # the first call autotunes the launch shape and sizes the capacity
        for j in range(0, len(cams), 4):
            r.use_device_cameras(table[j:j + 4].reshape(-1))
            for i, im in enumerate(r(*[P0[k] for k in names])):
                targets[j + i].copy_(im)
        assert not r.overflowed()
    extent = 1.1 * 6.0
    lrs = {"means": 1.6e-4 * extent, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2,
           "sh": 2.5e-3}
    rng = np.random.default_rng(7)
    picks = torch.from_numpy(np.stack([rng.choice(len(cams), 4, replace=False)
                                       for _ in range(steps)])).to(dev)
    nb = gsmi.ssim_workspace_bytes(3, 1080, 1920)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    # the step's inputs that change from step to step, at fixed addresses
    pick = picks[0].clone()
    cam_static = table.index_select(0, pick).reshape(-1).clone()
    r.use_device_cameras(cam_static)

    def start():
        gen = torch.Generator(device=dev)
        gen.manual_seed(6)
        P = {k: P0[k].clone() for k in names}
        P["means"] += 0.01 * torch.randn(P["means"].shape, device=dev, generator=gen)
        P["sh"][0] += 0.1 * torch.randn(P["sh"][0].shape, device=dev, generator=gen)
        for t in P.values():
            t.requires_grad_()
        mom = {k: (torch.zeros_like(P[k]), torch.zeros_like(P[k])) for k in names}
        return P, mom, gsmi.adam_counter(dev)

    def step(P, mom, counter, fused):
        cam_static.copy_(table.index_select(0, pick).reshape(-1))
        imgs = r(*[P[k] for k in names])
        tg = targets.index_select(0, pick)
        loss = sum(photometric_loss(im, tg[i], 0.2, ws) for i, im in enumerate(imgs)) / 4
        loss.backward()
        # with the Adam step fused into the backward, the optimiser launch only
        # advances the step counter
        opt = [] if fused else names
        gsmi.adam_step([(P[k].data, P[k].grad, mom[k][0], mom[k][1], lrs[k]) for k in opt],
                       sc.n, counter, tiles_touched=r.frame.buffer(gsmi.BUF_TILES_TOUCHED),
                       n_views=4)
        return loss.detach()

    def run(mode, fused=True):
        P, mom, counter = start()
        r.fuse_adam(gsmi.FusedAdamStep(mom, lrs, counter) if fused else None)
        losses = torch.zeros(steps, device=dev)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        graph = loss_static = None
        torch.cuda.synchronize()
        for s in range(steps):
            if mode == "graph" and s == warm:
                # capture after `warm` eager steps (run on a side stream, as capture wants)
                torch.cuda.synchronize()
                for t in P.values():
                    t.grad = None
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(graph):
                    loss_static = step(P, mom, counter, fused)
            ev[s][0].record()
            pick.copy_(picks[s])
            if graph is not None:
                graph.replay()
                losses[s].copy_(loss_static)
            else:
                for t in P.values():
                    t.grad = None
                if mode == "graph":
                    side = torch.cuda.Stream()
                    side.wait_stream(torch.cuda.current_stream())
                    with torch.cuda.stream(side):
                        losses[s] = step(P, mom, counter, fused)
                    torch.cuda.current_stream().wait_stream(side)
                else:
                    losses[s] = step(P, mom, counter, fused)
            ev[s][1].record()
        torch.cuda.synchronize()
        if r.overflowed():
            raise RuntimeError("instance capacity overflowed during the 6M training run (%s)" % mode)
        if int(counter[0]) != steps:
            raise RuntimeError("Adam counted %d steps of %d" % (int(counter[0]), steps))
        ms = [a.elapsed_time(b) for a, b in ev][first_timed - 1:]
        ls = losses.cpu().numpy()
        del graph, P, mom
        return {"mean_ms_per_step": round(float(np.mean(ms)), 4),
                "median_ms_per_step": round(float(np.median(ms)), 4),
                "first_loss": round(float(ls[0]), 6), "last_loss": round(float(ls[-1]), 6),
                "mean_loss_first_10": round(float(ls[:10].mean()), 6),
                "mean_loss_last_10": round(float(ls[-10:].mean()), 6)}

    eager = run("eager")
    log("6M training, eager: %.3f ms/step" % eager["mean_ms_per_step"])
    captured = run("graph")
    log("6M training, captured step: %.3f ms/step" % captured["mean_ms_per_step"])
    separate = run("eager", fused=False)
    log("6M training, eager, Adam as a separate launch: %.3f ms/step" % separate["mean_ms_per_step"])
    r.fuse_adam(None)
    nv, ni, _ = r.frame.status()
    out = {"workload": "6,000,000 Gaussians (64 spheres, 16 planes), SH3, 64 ring cameras at "
                       "1920x1080, 4 random views per step, autograd fwd+bwd + Eq. 3 loss "
                       "(L1 + 0.2 D-SSIM) + sparse Adam, from a perturbed copy",
           "gaussian_order": "spatial (Morton) order, as the trainer keeps it",
           "spatial_reorder": reorder,
           "steps": steps, "timed_steps": "%d..%d" % (first_timed, steps)}
    out.update(eager)
    out["optimizer"] = ("sparse Adam fused into the projection adjoint (gs_project_backward_adam); "
                        "a gs_adam_step_counted launch with no arrays advances the step count")
    out["captured"] = dict(captured, replayed_from_step=warm + 1)
    out["separate_adam"] = separate
    out.update({"visible_entries_last_step": nv, "instances_last_step": ni,
                "capacity": r.frame.cap, "tuned": r.tuned})
    del r, targets
    torch.cuda.empty_cache()
    return out, sc, cams


def calibration_copy(torch, dev):
    """A plain device copy of known size (256 MiB read + 256 MiB written): the
    reference that scales rocprofv3's HBM byte counters in a profiled run."""
    src = torch.ones(64 << 20, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def profile_workload(args):
    """One of the secondary workloads alone, with a fixed launch shape (no
    tuner runs in the trace)."""
    import numpy as np
    import torch
    from paper_2507_20239_amd import gsmi, synth
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    shape = {"raster_batch": args.raster_batch, "persistent_blocks": args.persistent,
             "depth_presort": args.presort, "balanced_digits": args.balanced, "lanes": args.lanes}
    if args.profile_workload in ("batched_8_views", "plain_128x128"):
        sb = synth.batched_c2f() if args.profile_workload == "batched_8_views" else synth.tiny_scene()
        pb, _ = spatially_ordered(torch, gsmi, to_dev(sb, dev, torch, gsmi), reps=1)
        st = Step(sb, sb.cameras, pb, gsmi.raster_opts(**shape), 32 << 20, torch, gsmi, dev)
        st.eager()
        st.checked()
        st.capture()
        ms = time_loop(torch, st.launch, K, W)
    else:
        from paper_2507_20239_amd.autograd import GaussianRasterizer
        sc = synth.procedural_scene()
        cams = synth.procedural_cameras()[:4]
        P = {k: torch.from_numpy(np.ascontiguousarray(getattr(sc, k))).to(dev)
             for k in gsmi.PARAM_NAMES}
        P, _ = spatially_ordered(torch, gsmi, P, reps=1)
        for t in P.values():
            t.requires_grad_()
        r = GaussianRasterizer(sc.n, cams, sc.sh_degree, device=dev, **shape)
        g = torch.Generator(device=dev)
        g.manual_seed(5)
        Ws = [torch.randn(3, c.height, c.width, device=dev, generator=g) * 1e-6 for c in cams]

        def step():
            for t in P.values():
                t.grad = None
            torch.autograd.backward(r(P["means"], P["log_scales"], P["quats"],
                                      P["opacity_logits"], P["sh"]), Ws)

        ms = timed(torch, step, K, W)
    calibration_copy(torch, dev)
    print(json.dumps({"workload": args.profile_workload, "ms_per_step": round(ms, 4),
                      "launch_shape": shape}), flush=True)


# ---------------------------------------------------------------------------------------
# CPU baseline: the FP64 oracle as it stands, on all cores and on one
# ---------------------------------------------------------------------------------------
def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _med3(fn):
    """(median seconds of 3 runs, last result)."""
    ts, res = [], None
    for _ in range(3):
        t0 = time.perf_counter()
        res = fn()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), res


def _subscene(sc, m):
    """The first m Gaussians of a scene (projection and chain-rule costs are
    linear in the Gaussian count, so a prefix is a fair sample)."""
    import types
    if m >= sc.n:
        return sc
    return types.SimpleNamespace(
        means=sc.means[:, :m], log_scales=sc.log_scales[:, :m], quats=sc.quats[:, :m],
        opacity_logits=sc.opacity_logits[:m], sh=sc.sh[..., :m], sh_degree=sc.sh_degree, n=m)


class OracleStep:
    """One training step's forward + backward by the FP64 oracle over a list of
    views, estimated from bounded samples: projection and chain rule of all
    Gaussians (on one thread: of a prefix of `one_sub` Gaussians, scaled), per-pixel
    compositing and its adjoint on random pixels (scaled to every pixel)."""

    def __init__(self, sc, cams, px_all, px_one, one_sub=200_000, render_views=None, seed=0):
        import numpy as np
        self.np = np
        self.sc, self.cams = sc, list(cams)
        self.px_all, self.px_one, self.one_sub = px_all, px_one, one_sub
        # views whose pixels are sampled (all of them unless stated; the others take the
        # per-pixel rates of the sampled ones)
        self.render_views = render_views if render_views is not None else list(range(len(cams)))
        self.rng = np.random.default_rng(seed)
        self.proj = {}

    def run(self, oracle, threads):
        np = self.np
        oracle.set_threads(threads)
        sc = self.sc
        one = threads == 1
        sub = _subscene(sc, self.one_sub) if one else sc
        scale_g = sc.n / sub.n
        t_proj = t_chain = 0.0
        fwd_rate, bwd_rate = [], []
        for v, cam in enumerate(self.cams):
            if v not in self.render_views and v > 0:
                t_proj += t_proj_v
                t_chain += t_chain_v
                continue
            tp, p_sub = _med3(lambda: oracle.project(sub, cam))
            t_proj_v = tp * scale_g
            t_proj += t_proj_v
            if v not in self.proj:
                self.proj[v] = p_sub if sub is sc else oracle.project(sc, cam)
            p = self.proj[v]
            m = self.px_one if one else self.px_all
            m = max(1, m // len(self.render_views))
            flat = self.rng.choice(cam.width * cam.height, size=m, replace=False)
            pix = np.stack([flat % cam.width, flat // cam.width], 1).astype(np.int32)
            g = self.rng.standard_normal((m, 3)) * 1e-3
            tf, _ = _med3(lambda: oracle.render_pixels(p, pix))
            tb, (gproj, _) = _med3(lambda: oracle.render_backward_pixels(p, pix, g))
            fwd_rate.append(tf / m)
            bwd_rate.append(tb / m)
            # chain rule: the sampled gradients stand in for the full image's (its cost
            # depends on the visible count, not on the values)
            if one:
                gs = gproj[:sub.n]
                tc, _ = _med3(lambda: oracle.project_backward(
                    sub, cam, p_sub["visible"], gs, stats=(np.zeros(sub.n), np.zeros(sub.n))))
            else:
                tc, _ = _med3(lambda: oracle.project_backward(
                    sc, cam, p["visible"], gproj, stats=(np.zeros(sc.n), np.zeros(sc.n))))
            t_chain_v = tc * scale_g
            t_chain += t_chain_v
        P = sum(c.width * c.height for c in self.cams)
        t_pix = (statistics.mean(fwd_rate) + statistics.mean(bwd_rate)) * P
        return t_proj + t_chain + t_pix

    def describe(self, threads_all):
        views = ("all %d views" % len(self.cams) if len(self.render_views) == len(self.cams)
                 else "view(s) %s (rates applied to all %d views)" % (self.render_views,
                                                                       len(self.cams)))
        return ("projection + chain rule of all %d Gaussians per view (%d threads; 1 thread: a "
                "prefix of %d Gaussians, scaled), compositing + adjoint on %d random pixels "
                "(%d threads) / %d pixels (1 thread) of %s, scaled to all pixels; median of 3 "
                "per component" % (self.sc.n, threads_all, min(self.one_sub, self.sc.n),
                                   self.px_all, threads_all, self.px_one, views))


def cpu_baseline(scenes, dens, dL_c1):
    """The FP64 oracle, untuned, timed on this host for each workload, on all
    threads and on one.  Returns the bench line's cpu_baseline object."""
    import numpy as np
    import oracle
    threads = oracle.max_threads()
    per = {}

    def both(fn):
        oracle.set_threads(threads)
        a, _ = _med3(fn)
        oracle.set_threads(1)
        b, _ = _med3(fn)
        oracle.set_threads(threads)
        return a, b

    # 128x128, 2,000 Gaussians: the whole step, exactly
    sc1 = scenes["c1"]
    cam1 = sc1.cameras[0]
    tgt1 = sc1.targets[0]

    def c1_step():
        p = oracle.project(sc1, cam1)
        C, T, nc, mg = oracle.render_image(p)
        _, dL = oracle.l1_loss_grad(C, tgt1)
        gproj, _ = oracle.render_backward_image(p, dL)
        oracle.project_backward(sc1, cam1, p["visible"], gproj,
                                stats=(np.zeros(sc1.n), np.zeros(sc1.n)))

    log("CPU oracle: 128x128 step")
    a, b = both(c1_step)
    per["plain_128x128_2k"] = {"all_threads_ms": round(a * 1e3, 2), "one_thread_ms": round(b * 1e3, 2),
                               "sampled": "no: the whole step"}
    # the sampled steps
    for key, sc, cams, px_all, px_one, views in (
            ("single_view_1m_1600x1040", scenes["c2"], scenes["c2"].cameras, 1024, 48, None),
            ("batched_8_views_500k", scenes["c3"], scenes["c3"].cameras, 1024, 64, None),
            ("step_6m_4x1920x1080", scenes["c5"], scenes["c5_cams"], 256, 16, [0])):
        if sc is None:
            continue
        log("CPU oracle: %s" % key)
        o = OracleStep(sc, cams, px_all, px_one, render_views=views)
        ta = o.run(oracle, threads)
        tb = o.run(oracle, 1)
        per[key] = {"all_threads_ms": round(ta * 1e3, 1), "one_thread_ms": round(tb * 1e3, 1),
                    "sampled": o.describe(threads)}
        del o
    # densification of 3M Gaussians: statistic over 100 views, selection, map, rows
    if dens is not None:
        log("CPU oracle: densification of 3M Gaussians")
        n = dens.means.shape[1]
        tg, tls, tlo = oracle.thresholds(2e-4, 0.01, dens.extent, 0.005)
        rng = np.random.default_rng(0)
        sh = rng.random((48, n), dtype=np.float32)
        params = {"means": dens.means, "log_scales": dens.log_scales, "quats": dens.quats,
                  "opacity_logits": dens.opacity_logits, "sh": sh}
        frac = 0.1
        n_pre = int(n * frac)
        # the rows' gather on the parents of a prefix: parameters and two moment arrays
        # of the same shapes (177 rows per Gaussian, as the GPU gathers)
        pre = {k: v[..., :n_pre] for k, v in params.items()}
        for k in list(params):
            pre["m_" + k] = pre[k]
            pre["v_" + k] = pre[k]

        def densify():
            acc, den = oracle.stats_f32(dens.dmean2d, dens.visible, dens.view_wh)
            s, c, p = oracle.select(acc, den, dens.log_scales, dens.opacity_logits, tg, tls, tlo)
            src, kind = oracle.densify_plan(s, c, p)
            m = int(np.searchsorted(src, n_pre))
            t0 = time.perf_counter()
            oracle.densify_apply(pre, src[:m], kind[:m], 0x5EED, 0)
            return time.perf_counter() - t0

        def timed_densify(th):
            oracle.set_threads(th)
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                t_apply = densify()
                total = time.perf_counter() - t0
                # the rows' gather timed on a tenth of the output rows, scaled
                ts.append(total - t_apply + t_apply / frac)
            return statistics.median(ts)

        a = timed_densify(threads)
        b = timed_densify(1)
        oracle.set_threads(threads)
        per["densify_3m_100_views"] = {
            "all_threads_ms": round(a * 1e3, 1), "one_thread_ms": round(b * 1e3, 1),
            "sampled": "statistic over all 100 views, selection and map of all 3M Gaussians in "
                       "full; the FP64 row gather (parameters with SH3 and two moment arrays, "
                       "Philox split means) for the parents among the first 10% of the "
                       "Gaussians, scaled by 10; median of 3"}
    main = per.get("single_view_1m_1600x1040") or per["plain_128x128_2k"]
    return {"value": main["all_threads_ms"], "unit": "ms per fwd+bwd iter (1M Gaussians, 1600x1040)",
            "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "nproc": os.cpu_count(),
            "sample": main["sampled"], "per_workload": per}


# ---------------------------------------------------------------------------------------
def main():
    args = parse()
    if args.profile_workload:
        profile_workload(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (sharding the views "
              "across GPUs is a design only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2507_20239_amd import gsmi, synth

    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup

    # ---------------- metric workload: 1M Gaussians, 1600x1040, SH3 ----------------
    log("generating 1M-Gaussian scene")
    sc = synth.single_view_1m()
    params0 = to_dev(sc, dev, torch, gsmi)
    # the generator's order (uniform random positions: the Gaussians a view renders are
    # scattered over the index range); a profiling run times the value's configuration only
    leg0 = leg1 = {"hbm": []}
    if not args.profile:
        leg0, st0 = metric_leg(torch, gsmi, sc, params0, dev, K, W, "generator order")
        del st0
    # the spatial order the trainer keeps (applied at every densification): the same
    # Gaussians permuted by gs_spatial_order + gs_densify_apply; its cost is reported
    params, reorder = spatially_ordered(torch, gsmi, params0)
    if not args.profile:
        leg1, st1 = metric_leg(torch, gsmi, sc, params, dev, K, W, "spatial order, dense gradients")
        del st1
    # the trainer's configuration: spatial order, gradient rows of rendered Gaussians
    leg, st = metric_leg(torch, gsmi, sc, params, dev, K, W, "spatial order, rendered rows",
                         rendered_only=True)
    ms, parts, roofline, hbm = leg["ms"], leg["breakdown_ms"], leg["roofline"], leg["hbm"]
    nvis, ninst = leg["visible"], leg["instances"]
    ms_graph, ms_eager = leg["graph_ms"], leg["eager_ms"]
    del params0

    if args.profile:
        calibration_copy(torch, dev)

    result = {
        "metric": "ms per fwd+bwd iter at 1M Gaussians 1600×1040; batched vs plain speedup",
        "value": round(ms, 4), "unit": "ms", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(ms, 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "single view 1600x1040, 1,000,000 Gaussians, SH degree 3, "
                               "fwd+bwd+densify statistic",
                   "launch": "hipGraph" if ms_graph <= ms_eager else "eager",
                   "gaussian_order": "spatial (Morton) order, as the trainer keeps it",
                   "gradients": "rows of the Gaussians the view rendered (sparse Adam's input; the "
                                "others are zero and not written)",
                   "gaussians": sc.n, "width": 1600, "height": 1040, "sh_degree": 3,
                   "visible": nvis, "instances": ninst},
        "graph_ms": round(ms_graph, 4), "eager_ms": round(ms_eager, 4),
        "breakdown_ms": {k: round(v, 4) for k, v in parts.items()},
        "roofline": roofline,
        "generator_order": {k: v for k, v in leg0.items() if k not in ("hbm",)},
        "spatial_order_dense_gradients": {k: v for k, v in leg1.items() if k not in ("hbm",)},
        "spatial_reorder": reorder,
    }
    scenes = {"c2": sc, "c3": None, "c5": None, "c5_cams": None}

    if not args.profile:
        log("plain 128x128 step")
        result["plain_128x128"], scenes["c1"] = plain_128(torch, gsmi, synth, dev, K, W)

    # ---------------- batched coarse-to-fine vs per-view plain ----------------
    if not args.no_batched and not args.profile:
        result["batched"], scenes["c3"] = batched_leg(torch, gsmi, synth, dev, K, W)

    # ---------------- the other steps of an iteration and of a densification ----------------
    dens = None
    if not args.no_extras and not args.profile:
        ex, hbm_x, dens = extras(torch, gsmi, synth, st, params, sc, dev)
        hbm += hbm_x
        result["extras"] = ex
        c5, scenes["c5"], cams5 = c5_training(torch, gsmi, synth, dev, args.c5_steps)
        scenes["c5_cams"] = cams5[:4]
        result["training_6m_4x1920x1080"] = c5
        log("6M training: %.3f ms/step, loss %.4f -> %.4f"
            % (c5["mean_ms_per_step"], c5["first_loss"], c5["last_loss"]))
    result["hbm_stages"] = hbm + [dict(h, stage=h["stage"] + " (generator order)")
                                  for h in leg0["hbm"]]

    # ---------------- CPU baseline: the FP64 oracle ----------------
    if not args.no_cpu and not args.profile:
        del st
        torch.cuda.empty_cache()
        result["cpu_baseline"] = cpu_baseline(scenes, dens, None)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
