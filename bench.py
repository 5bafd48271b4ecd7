#!/usr/bin/env python3
"""Block-matching throughput on one MI355X: ref-patches/s and per-step latency.

Workload: one 512x512 grayscale float32 image (Voronoi cells + noise sigma 50/255, seed 1),
8x8 patches, reference stride 3, 39x39 search window, K = 16 -- 28,561 references and
41,615,401 in-window pairs per step.  A step is the whole path on the resident image:
the patch-norm box filter (bm_norms) followed by the fused cross-term / distance / top-K
kernel (bm_cross_topk); the two calls together are exactly bm_match.

Output: one JSON line.  Every precision form is timed (plain float32, bfloat16 split,
float16 split); `value` is ref-patches/s of the reported form (default: the bfloat16 split,
whose distances are exactly those of the image rounded to 16 significant bits, the form
of the serving workload) over the timed region with the inputs already in HBM, and
`plain_fp32` gives the plain float32 form beside it.  `roofline` covers the dominant
kernel (the cross-term kernel of the reported form), timed with HIP events on its own
launch stream, against the published
matrix peak and the peak measured in the same run (`peaks_measured`: a matrix-op loop per
form and a streaming copy); `executed` adds the matrix/vector pipe utilisation from the
committed counter summary when it matches the current sources.  The same line carries
short forms of the other workloads: `rgbnir1024` (the split-precision workload, 1024 x
1024 x 4 with joint 8 x 8 x 4 patches, every form, with its accuracy), `shapes` (the
paper's single-channel runtime setup, 6 x 6 patches at stride 1 in a 30 x 30 window, every
form with its accuracy, and a window outside the specialised envelope on the generic
float32 kernel), `batch64` (the
64-image uneven batch, one bm_match_batch call per step in each form, and the same images
as 64 bm_match calls), `serving` (Poisson streams through bm_submit / bm_poll at two
request rates, bfloat16 split; `latency_ms` then holds the request latency of the lower
rate), and `cpu_baseline`
(the FP64 oracle on this host: one core on a bounded sample, all cores on the whole
image) with `accuracy`, the error of every form against the oracle on a seeded sample.

Other workloads (not the headline line; one JSON line each):
  --workload batch64   64 images of uneven shapes (sides 128..1024, C in {1,3}, P in {6,8})
                       through bm_match_batch, against 64 single-image bm_match calls.
  --workload serving   Poisson request streams at the --qps rates (sides log-uniform in
                       [256, 2048], 1..4 channels) through bm_submit / bm_poll: achieved
                       ref-patches/s and p50/p99 request latency per rate.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ref patches/s (top-16, 8x8 patch, 39x39 window) vs plain FP32; p50/p99 latency"
PEAK_TFLOPS = {"fp32": 157.3, "bf16x4": 2500.0, "fp16x3": 2500.0}  # dense matrix-core peaks
DTYPE = {"fp32": "f32", "bf16x4": "bf16x4->f32", "fp16x3": "f16x3->f32"}
_FAST = ["xcorr_fast.h", "xcorr_lane.h", "xcorr_common.h", "contract.h", "select.h", "topk.h",
         "bm_internal.h", "split16.h"]
KERNEL_SOURCES = {"fp32": _FAST, "bf16x4": _FAST, "fp16x3": _FAST}


def source_hash(prec: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[prec]:
        p = os.path.join(ROOT, "paper_2006_13714_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def pair_count(H, W, P, s, Wn):
    """In-window (reference, candidate) pairs: the clipped window is separable per axis."""
    r = Wn // 2

    def axis(n):
        nv = n - P + 1
        return sum(min(nv - 1, c + r) - max(0, c - r) + 1 for c in range(0, nv, s))

    return axis(H) * axis(W)


def traffic_from_profile(prec: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it matches this source."""
    path = os.path.join(ROOT, "profiles", f"xcorr_{prec}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != source_hash(prec):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_refs(args):
    """Worker of the all-core oracle timing: the FP64 oracle on one slice of references."""
    img, P, s_, Wn, K, refs = args
    from oracle import bm_oracle as O
    O.bm(img, P, s_, Wn, K, refs=refs)
    return len(refs)


def cpu_baseline(img, sh, budget_s: float, forms=None, extra=None):
    """FP64 oracle timed on this host, and the accuracy of every GPU form against it.

    One core: every second reference in row-major order until budget_s has passed.  All
    cores: every reference of the image, sliced over a process pool of one worker per
    available core (workers started and warmed before the timed map).  Accuracy: the
    oracle's rows for a seeded sample of references, against each form's result (tolerance
    rule 1e-4 with the 1e-2 (N_i + N_j) floor; set rule).  `extra` maps another workload's
    name to (image, shape, {form: (idx, dist)}); its accuracy is reported the same way on
    a seeded sample plus the first and last reference rows and columns."""
    import multiprocessing as mp
    import numpy as np
    from oracle import bm_oracle as O

    n_ref = sh.n_ref
    sample = np.arange(0, n_ref, 2)
    done = 0
    t0 = time.perf_counter()
    for start in range(0, len(sample), 256):
        O.bm(img, sh.patch, sh.stride, sh.window, sh.k, refs=sample[start:start + 256])
        done += len(sample[start:start + 256])
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    out = {"value": done / dt, "unit": "ref-patches/s", "cores": 1, "kind": "oracle",
           "sample": f"{done} of {n_ref} references (every 2nd, row-major) of the same "
                     f"512x512 image, numpy float64 brute force, {dt:.1f} s on one core",
           "host_threads_available": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            out["cpu_model"] = next((l.split(":", 1)[1].strip() for l in f
                                     if l.startswith("model name")), None)
    except OSError:
        pass
    cores = min(16, len(os.sched_getaffinity(0)))
    if cores > 1:
        ctx = mp.get_context("spawn")
        pool = ctx.Pool(cores)
        try:
            refs = np.arange(n_ref)
            chunks = np.array_split(refs, cores * 4)
            pool.map_async(_oracle_refs, [(img, sh.patch, sh.stride, sh.window, sh.k, c[:1])
                                          for c in chunks[:cores]]).get(timeout=120)
            t0 = time.perf_counter()
            n = sum(pool.map_async(_oracle_refs, [(img, sh.patch, sh.stride, sh.window, sh.k, c)
                                                  for c in chunks]).get(timeout=300))
            dta = time.perf_counter() - t0
            out["all_cores"] = {"value": n / dta, "unit": "ref-patches/s", "cores": cores,
                                "sample": f"all {n} references of the image over {cores} "
                                          f"worker processes, {dta:.1f} s"}
        except Exception as e:  # a pool problem must not cost the benchmark line
            out["all_cores"] = {"error": repr(e)}
        finally:
            pool.terminate()
            pool.join()
    if forms:
        from tests import parity
        rng = np.random.default_rng(11)
        refs = np.unique(np.concatenate([rng.choice(n_ref, 1000, replace=False),
                                         np.arange(169), np.arange(n_ref - 169, n_ref)]))
        head = parity.OracleHead(img, sh.patch, sh.stride, sh.window, sh.k, refs=refs)
        acc = {}
        for f, (idx, dist) in forms.items():
            rep = head.check(idx[refs], dist[refs])
            r = rep.summary()
            r["within_rule"] = rep.tolerant_mismatch == 0 and rep.order_violations == 0
            acc[f] = r
        out["accuracy"] = {"refs": int(len(refs)),
                           "sample": "1000 seeded references (seed 11) plus the first and "
                                     "last reference rows", "forms": acc}
    for name, (ximg, xsh, xforms) in (extra or {}).items():
        from tests import parity
        nry = (xsh.height - xsh.patch) // xsh.stride + 1
        nrx = (xsh.width - xsh.patch) // xsh.stride + 1
        grid = np.arange(xsh.n_ref).reshape(nry, nrx)
        rng = np.random.default_rng(12)
        refs = np.unique(np.concatenate([rng.choice(xsh.n_ref, 600, replace=False),
                                         grid[0], grid[-1], grid[:, 0], grid[:, -1]]))
        t0 = time.perf_counter()
        head = parity.OracleHead(ximg, xsh.patch, xsh.stride, xsh.window, xsh.k, refs=refs)
        acc = {}
        for f, (idx, dist) in xforms.items():
            rep = head.check(idx[refs], dist[refs])
            r = rep.summary()
            r["within_rule"] = rep.tolerant_mismatch == 0 and rep.order_violations == 0
            acc[f] = r
        out.setdefault("accuracy_other", {})[name] = {
            "refs": int(len(refs)), "oracle_s": time.perf_counter() - t0,
            "sample": "600 seeded references (seed 12) plus every border reference",
            "forms": acc}
    return out


# Untimed warm-up floor per measured form: the device's clocks rise over the first tens of
# milliseconds under load, so a few warm-up steps alone leave the first timed steps slower.
WARM_S = 0.1


def warm(torch, step, warmup):
    """`warmup` untimed steps, then more (synchronised every 8) until WARM_S has passed."""
    t0 = time.perf_counter()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    while time.perf_counter() - t0 < WARM_S:
        for _ in range(8):
            step()
        torch.cuda.synchronize()


def run_form(bm, torch, img_t, sh, prec, steps, warmup, flags=0):
    desc = bm.make_desc(sh.height, sh.width, sh.channels, sh.patch, sh.stride, sh.window,
                        sh.k, prec, flags)
    plan = bm.bm_plan(desc)
    dev = img_t.device
    nrm = torch.empty(((sh.height - sh.patch + 1) * (sh.width - sh.patch + 1),),
                      dtype=torch.float32, device=dev)
    idx = torch.empty((plan.n_ref, sh.k), dtype=torch.int32, device=dev)
    dist = torch.empty((plan.n_ref, sh.k), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        bm.bm_norms(plan, img_t, nrm, stream)
        bm.bm_cross_topk(plan, img_t, nrm, idx, dist, stream)

    warm(torch, step, warmup)
    # throughput: `steps` steps back to back, bracketed by device synchronisations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-kernel and per-step times: the same steps again with HIP events between the calls
    # (the event markers cost device time of their own, so they stay out of the timed pass)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for i in range(steps):
        ev[i][0].record(stream)
        bm.bm_norms(plan, img_t, nrm, stream)
        ev[i][1].record(stream)
        bm.bm_cross_topk(plan, img_t, nrm, idx, dist, stream)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    norm_ms = [a.elapsed_time(b) for a, b, _ in ev]
    xc_ms = [b.elapsed_time(c) for _, b, c in ev]
    step_ms = [a.elapsed_time(c) for a, _, c in ev]
    return plan, wall, norm_ms, xc_ms, step_ms, (idx, dist)


NLM_B = 2.2  # ~ sqrt(2 sigma^2 n) for the gray512 noise (sigma 50/255, n = 64)


def run_nlm(bm, torch, img_t, sh, steps, warmup):
    """bm_nlm on the same workload (norms + NLM kernel per step): throughput from steps back
    to back, kernel times from a second pass with events."""
    desc = bm.make_desc(sh.height, sh.width, sh.channels, sh.patch, sh.stride, sh.window,
                        sh.k, "fp32")
    plan = bm.bm_plan(desc)
    dev = img_t.device
    patch = torch.empty((plan.n_ref, sh.channels, sh.patch, sh.patch), dtype=torch.float32,
                        device=dev)
    theta = torch.empty((plan.n_ref,), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    warm(torch, lambda: bm.bm_nlm(plan, img_t, NLM_B, patch, theta, None, stream), warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bm.bm_nlm(plan, img_t, NLM_B, patch, theta, None, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        bm.bm_nlm(plan, img_t, NLM_B, patch, theta, None, stream)
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev], wall


def run_groups(bm, torch, img_t, sh, idx, steps):
    """bm_gather and bm_aggregate of the K-groups of the reported form's result."""
    plan = bm.cached_plan(bm.make_desc(sh.height, sh.width, sh.channels, sh.patch, sh.stride,
                                       sh.window, sh.k, "fp32"))
    dev = img_t.device
    groups = torch.empty((plan.n_ref, sh.k, sh.channels, sh.patch, sh.patch),
                         dtype=torch.float32, device=dev)
    out = torch.empty_like(img_t)
    ws = torch.empty((bm.bm_aggregate_workspace(plan),), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        bm.bm_gather(plan, img_t, idx, groups, stream)
        bm.bm_aggregate(plan, groups, idx, out, ws, stream)

    warm(torch, step, 1)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for a, b, c in ev:
        a.record(stream)
        bm.bm_gather(plan, img_t, idx, groups, stream)
        b.record(stream)
        bm.bm_aggregate(plan, groups, idx, out, ws, stream)
        c.record(stream)
    torch.cuda.synchronize()
    g_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    a_ms = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    gbytes = groups.numel() * 4
    return {"gather_ms": g_ms, "aggregate_ms": a_ms, "group_bytes": gbytes,
            "gather_write_GBps": gbytes / g_ms / 1e6, "aggregate_read_GBps": gbytes / a_ms / 1e6}


def run_volume(bm, torch, w, prec, steps, warmup):
    """3D search (window_depth > 0) on a synthetic volume: bm_norms (one map per slab) +
    bm_cross_topk per step, timed with events on the launch stream."""
    sh = w.shape
    desc = bm.make_desc(sh.height, sh.width, sh.planes, sh.patch, sh.stride, sh.window, sh.k,
                        prec, 0, sh.patch_depth, sh.window_depth)
    plan = bm.bm_plan(desc)
    dev = torch.device("cuda:0")
    vol = torch.from_numpy(w.image).to(dev)
    Z = sh.planes - sh.patch_depth + 1
    nrm = torch.empty((Z, sh.height - sh.patch + 1, sh.width - sh.patch + 1),
                      dtype=torch.float32, device=dev)
    idx = torch.empty((plan.n_ref, sh.k), dtype=torch.int32, device=dev)
    dist = torch.empty((plan.n_ref, sh.k), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        bm.bm_norms(plan, vol, nrm, stream)
        bm.bm_cross_topk(plan, vol, nrm, idx, dist, stream)

    warm(torch, step, warmup)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b, c in ev:
        a.record(stream)
        bm.bm_norms(plan, vol, nrm, stream)
        b.record(stream)
        bm.bm_cross_topk(plan, vol, nrm, idx, dist, stream)
        c.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    xc = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    nm = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    # pairs: every reference depth's clipped depth window times the clipped 2D window
    slabs = sum(min(Z - 1, z - (sh.window_depth - 1) // 2 + sh.window_depth - 1)
                - max(0, z - (sh.window_depth - 1) // 2) + 1 for z in range(Z))
    pairs = slabs * pair_count(sh.height, sh.width, sh.patch, sh.stride, sh.window)
    flops = 2.0 * sh.patch * sh.patch * sh.patch_depth * pairs
    return {"value": plan.n_ref * steps / wall, "unit": "ref-patches/s",
            "ms_per_step": wall / steps * 1e3, "norms_ms": nm, "cross_topk_ms": xc,
            "pairs_per_s": pairs / (xc / 1e3), "roofline_frac": flops / (xc / 1e3) / 1e12 / PEAK_TFLOPS[prec],
            "config": bm.bm_plan_config(plan)[0]}


def volumes(bm, synth, torch, steps, warmup):
    out = {}
    for make in (synth.video20, synth.multimodal6):
        w = make()
        sh = w.shape
        out[w.name] = {"shape": {"planes": sh.planes, "height": sh.height, "width": sh.width,
                                 "patch": sh.patch, "patch_depth": sh.patch_depth,
                                 "stride": sh.stride, "window": sh.window,
                                 "window_depth": sh.window_depth, "k": sh.k,
                                 "n_ref": sh.n_ref, "seed": w.seed}}
        for prec in ("fp32", "fp16x3"):
            out[w.name][prec] = run_volume(bm, torch, w, prec, steps, warmup)
    return out


def quantile(v, q):
    s = sorted(v)
    k = min(len(s) - 1, max(0, int(round(q * (len(s) - 1)))))
    return s[k]


# sub-measurements of the default line besides the three gray512 forms
SECTIONS = ["ncc", "nlm", "groups", "volumes", "rgbnir", "shapes", "peaks", "batch", "serving",
            "cpu"]


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--warm-ms", type=float, default=100.0,
                    help="untimed warm-up floor per measured form (clock ramp-up)")
    ap.add_argument("--precision", default="bf16x4", choices=list(PEAK_TFLOPS))
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle work for the CPU baseline (0 disables it)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 64 MiB device copy (counter calibration)")
    ap.add_argument("--workload", default="gray512", choices=["gray512", "batch64", "serving"])
    ap.add_argument("--batch-max-side", type=int, default=1024,
                    help="batch64: largest image side (sides uniform in [128, this])")
    ap.add_argument("--qps", default="50,200,500,1000,2000",
                    help="serving: comma-separated request rates")
    ap.add_argument("--serve-seconds", type=float, default=4.0,
                    help="serving: length of each rate's request stream")
    ap.add_argument("--clients", type=int, default=4,
                    help="serving: client threads sharing the request stream")
    ap.add_argument("--batch-steps", type=int, default=3,
                    help="default line: timed calls of the 64-image batch per form (0: skip)")
    ap.add_argument("--serve-seconds-default", type=float, default=2.0,
                    help="default line: length of each serving rate's stream (0: skip)")
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="default line: sub-measurements to run besides the three gray512 "
                         "forms (comma-separated subset of " + ",".join(SECTIONS) + "; a "
                         "profiler run can keep to the kernels it summarises)")
    args = ap.parse_args()
    sections = set(x for x in args.sections.split(",") if x)
    unknown = sections - set(SECTIONS)
    if unknown:
        ap.error(f"unknown sections {sorted(unknown)}")
    global WARM_S
    WARM_S = max(0.0, args.warm_ms) / 1e3

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; multi-GPU runs are not part of it "
              "(the repository's design notes describe how the path would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_13714_amd import bm, synth

    if not os.path.exists(bm.LIB_PATH):
        from paper_2006_13714_amd import build_lib
        build_lib.build()
    if args.workload == "batch64":
        return bench_batch(args, bm, synth, torch)
    if args.workload == "serving":
        return bench_serving(args, bm, synth, torch)

    w = synth.gray512()
    sh = w.shape
    img_t = torch.from_numpy(w.image).to("cuda:0")

    if args.calib_copy:
        src = torch.ones(16 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()

    results = {}
    for prec in ["fp32", "bf16x4", "fp16x3"]:
        results[prec] = run_form(bm, torch, img_t, sh, prec, args.steps, args.warmup)
    # the same workload ranked by normalized cross-correlation (BM_FLAG_NCC)
    ncc = {}
    if "ncc" in sections:
        for prec in ["fp32", "fp16x3"]:
            ncc[prec] = run_form(bm, torch, img_t, sh, prec, args.steps, args.warmup,
                                 bm.BM_FLAG_NCC)
    nlm_res = run_nlm(bm, torch, img_t, sh, args.steps, args.warmup) if "nlm" in sections else None
    grp = (run_groups(bm, torch, img_t, sh, results[args.precision][5][0], min(args.steps, 50))
           if "groups" in sections else None)

    prec = args.precision
    plan, wall, norm_ms, xc_ms, step_ms, _ = results[prec]
    n_ref = plan.n_ref
    value = n_ref * args.steps / wall
    pairs = pair_count(sh.height, sh.width, sh.patch, sh.stride, sh.window)
    flops = 2.0 * sh.patch * sh.patch * sh.channels * pairs
    xc_avg_s = sum(xc_ms) / len(xc_ms) / 1e3
    achieved = flops / xc_avg_s / 1e12
    peak = PEAK_TFLOPS[prec]
    traffic = traffic_from_profile(prec, w.name)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ref-patches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warm_floor_ms": args.warm_ms,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": w.name, "height": sh.height, "width": sh.width,
                   "channels": sh.channels, "patch": sh.patch, "stride": sh.stride,
                   "window": sh.window, "k": sh.k, "precision": prec, "n_ref": n_ref,
                   "pairs": pairs, "seed": w.seed},
        "latency_ms": {"p50": quantile(step_ms, 0.5), "p99": quantile(step_ms, 0.99),
                       "norm_avg": sum(norm_ms) / len(norm_ms),
                       "cross_topk_avg": xc_avg_s * 1e3},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": f"xcorr_topk ({prec})",
                     "algorithmic_flops_per_launch": flops},
    }
    forms = {}
    for f, (pf, wf, nf, xf, sf, _) in results.items():
        xa = sum(xf) / len(xf) / 1e3
        forms[f] = {"value": pf.n_ref * args.steps / wf, "ms_per_step": wf / args.steps * 1e3,
                    "cross_topk_ms": xa * 1e3, "p50_ms": quantile(sf, 0.5),
                    "p99_ms": quantile(sf, 0.99), "config": bm.bm_plan_config(pf)[0],
                    "roofline_frac": flops / xa / 1e12 / PEAK_TFLOPS[f]}
    out["forms"] = forms
    if nlm_res is not None:
        nlm_ms, nlm_wall = nlm_res
        nlm_flops = 2 * flops  # cross term + weighted patch sum, per in-window pair
        out["nlm"] = {"value": sh.n_ref * args.steps / nlm_wall, "unit": "ref-patches/s",
                      "ms_per_step": nlm_wall / args.steps * 1e3, "b": NLM_B,
                      "kernel_ms": sum(nlm_ms) / len(nlm_ms),
                      "roofline_frac": nlm_flops / (sum(nlm_ms) / len(nlm_ms) / 1e3) / 1e12 /
                      PEAK_TFLOPS["fp32"]}
    if grp is not None:
        out["groups"] = grp
    if ncc:
        out["ncc_forms"] = {
            f: {"value": pf.n_ref * args.steps / wf, "cross_topk_ms": sum(xf) / len(xf),
                "p50_ms": quantile(sf, 0.5), "p99_ms": quantile(sf, 0.99)}
            for f, (pf, wf, nf, xf, sf, _) in ncc.items()}
    if "volumes" in sections:
        out["volumes"] = volumes(bm, synth, torch, max(3, args.steps // 20), 2)
    rgb_outs = None
    if "rgbnir" in sections:
        rgb, rgb_outs = rgbnir_summary(bm, synth, torch, max(5, args.steps // 10))
        out["rgbnir1024"] = rgb
    shape_outs = None
    if "shapes" in sections:
        shp, shape_outs = shapes_summary(bm, synth, torch, img_t, w.image, max(5, args.steps // 10))
        out["shapes"] = shp
    # measured attainable peaks beside the published ones
    if "peaks" in sections:
        peaks = {f: bm.bm_peak_mfma(f, 0) for f in PEAK_TFLOPS}
        peaks32 = {f: bm.bm_peak_mfma(f, 1) for f in PEAK_TFLOPS}
        copy_gbps = bm.bm_peak_copy(1 << 30, 5)
        out["peaks_measured"] = {"mfma_tflops": peaks, "mfma_32x32_tflops": peaks32,
                                 "copy_GBps": copy_gbps,
                                 "published": {"mfma_tflops": PEAK_TFLOPS, "hbm_GBps": 8000.0}}
        out["roofline"]["peak_measured"] = peaks[prec]
        out["roofline"]["frac_measured"] = achieved / peaks[prec]
        for f in forms:
            forms[f]["roofline_frac_measured"] = (forms[f]["roofline_frac"] * PEAK_TFLOPS[f] /
                                                  peaks[f])
    counters = mfma_busy_from_profile(prec, w.name)
    if counters is not None:
        out["roofline"]["executed"] = counters
    out["norm"] = {"ms": sum(norm_ms) / len(norm_ms),
                   "algorithmic_bytes": 4.0 * sh.height * sh.width * sh.channels +
                   4.0 * (sh.height - sh.patch + 1) * (sh.width - sh.patch + 1)}
    out["norm"]["GBps"] = out["norm"]["algorithmic_bytes"] / (out["norm"]["ms"] * 1e6)
    # the uneven 64-image batch and the serving loop, short forms of their own workloads
    if args.batch_steps > 0 and "batch" in sections:
        out["batch64"] = batch_summary(bm, synth, torch, args.batch_steps)
    if args.serve_seconds_default > 0 and "serving" in sections:
        pool = [w_ for _, w_ in synth.serving_requests(16, 100.0)]
        sweep = serve_sweep(bm, pool, SERVE_FORM, SERVE_QPS, args.serve_seconds_default,
                            args.clients)
        out["serving"] = {"precision": SERVE_FORM, "pool": len(pool), "clients": args.clients,
                          "sides": "log-uniform 256..2048", "channels": "1..4",
                          "latency": "submit to results in host memory (PCIe copies included)",
                          "sweep": sweep}
        low = sweep[0]
        out["latency_ms"] = {"p50": low["p50_ms"], "p99": low["p99_ms"],
                             "kind": f"serving request latency at {low['qps']:.0f} requests/s "
                                     f"({SERVE_FORM})",
                             "step_p50": quantile(step_ms, 0.5),
                             "step_p99": quantile(step_ms, 0.99),
                             "norm_avg": sum(norm_ms) / len(norm_ms),
                             "cross_topk_avg": xc_avg_s * 1e3}
    v32 = forms["fp32"]["value"]
    out["plain_fp32"] = {"value": v32, "speedup": value / v32}
    if args.cpu_budget > 0 and "cpu" in sections:
        outs = {f: (r[5][0].cpu().numpy(), r[5][1].cpu().numpy()) for f, r in results.items()}
        extra = {}
        if rgb_outs:
            extra["rgbnir1024"] = rgb_outs
        if shape_outs:
            extra["paper_setup"] = shape_outs
        out["cpu_baseline"] = cpu_baseline(w.image, sh, args.cpu_budget, outs, extra)
        acc = out["cpu_baseline"].get("accuracy", {}).get("forms", {})
        out["accuracy"] = acc
        other = out["cpu_baseline"].get("accuracy_other", {})
        if "rgbnir1024" in other:
            out["rgbnir1024"]["accuracy"] = other["rgbnir1024"]
        if "paper_setup" in other:
            out["shapes"]["paper_setup"]["accuracy"] = other["paper_setup"]
        if prec in acc and not acc[prec]["within_rule"]:
            out["plain_fp32"]["speedup"] = None
            out["plain_fp32"]["note"] = f"{prec} is outside the 1e-4 rule on the sample"
    print(json.dumps(out), flush=True)


def shapes_summary(bm, synth, torch, img_t, img, steps):
    """Two more shapes on the gray512 image: the paper's single-channel runtime setup
    (6 x 6 patches, stride 1, 30 x 30 window, Sec. V-A; K = 16) in every form, and a shape
    outside the specialised kernel's envelope (8 x 8 patches, stride 3, 61 x 61 window:
    3 s + Wn = 70 > 48), which runs the generic float32 kernel.  Returns the summary and the
    paper setup's outputs (for accuracy)."""
    res = {}
    outs = {}
    for name, (P, s_, Wn, forms) in {"paper_setup": (6, 1, 30, ["fp32", "bf16x4", "fp16x3"]),
                                     "generic_fp32": (8, 3, 61, ["fp32"])}.items():
        sh = synth.BMShape(512, 512, 1, P, s_, Wn, 16)
        pairs = pair_count(sh.height, sh.width, P, s_, Wn)
        flops = 2.0 * P * P * pairs
        entry = {"height": 512, "width": 512, "channels": 1, "patch": P, "stride": s_,
                 "window": Wn, "k": 16, "n_ref": sh.n_ref, "pairs": pairs, "forms": {}}
        for prec in forms:
            plan, wall, norm_ms, xc_ms, step_ms, (idx, dist) = run_form(
                bm, torch, img_t, sh, prec, steps, 2)
            xa = sum(xc_ms) / len(xc_ms) / 1e3
            entry["forms"][prec] = {"value": sh.n_ref * steps / wall,
                                    "ms_per_step": wall / steps * 1e3,
                                    "cross_topk_ms": xa * 1e3,
                                    "config": bm.bm_plan_config(plan)[0],
                                    "roofline_frac": flops / xa / 1e12 / PEAK_TFLOPS[prec]}
            if name == "paper_setup":
                outs[prec] = (idx.cpu().numpy(), dist.cpu().numpy())
        res[name] = entry
    return res, (img, synth.BMShape(512, 512, 1, 6, 1, 30, 16), outs)


def rgbnir_summary(bm, synth, torch, steps):
    """The split-precision workload (1024 x 1024 x 4, joint 8 x 8 x 4 patches, stride 4,
    31 x 31 window, K = 32): every form timed as in the headline (bm_norms + bm_cross_topk
    per step, HIP events); returns the summary and each form's outputs (for accuracy)."""
    w = synth.rgbnir1024()
    sh = w.shape
    img_t = torch.from_numpy(w.image).to("cuda:0")
    pairs = pair_count(sh.height, sh.width, sh.patch, sh.stride, sh.window)
    flops = 2.0 * sh.patch * sh.patch * sh.channels * pairs
    res = {"workload": w.name, "height": sh.height, "width": sh.width,
           "channels": sh.channels, "patch": sh.patch, "stride": sh.stride,
           "window": sh.window, "k": sh.k, "n_ref": sh.n_ref, "pairs": pairs,
           "algorithmic_flops": flops, "forms": {}}
    outs = {}
    for prec in ["fp32", "bf16x4", "fp16x3"]:
        plan, wall, norm_ms, xc_ms, step_ms, (idx, dist) = run_form(
            bm, torch, img_t, sh, prec, steps, 2)
        xa = sum(xc_ms) / len(xc_ms) / 1e3
        res["forms"][prec] = {"value": sh.n_ref * steps / wall,
                              "ms_per_step": wall / steps * 1e3, "cross_topk_ms": xa * 1e3,
                              "norm_ms": sum(norm_ms) / len(norm_ms),
                              "config": bm.bm_plan_config(plan)[0],
                              "roofline_frac": flops / xa / 1e12 / PEAK_TFLOPS[prec]}
        outs[prec] = (idx.cpu().numpy(), dist.cpu().numpy())
    v32 = res["forms"]["fp32"]["value"]
    for prec in res["forms"]:
        res["forms"][prec]["speedup_vs_fp32"] = res["forms"][prec]["value"] / v32
    return res, (w.image, sh, outs)


SERVE_FORM = "bf16x4"
SERVE_QPS = [200.0, 800.0]


def batch_summary(bm, synth, torch, steps):
    """The 64-image uneven batch: one bm_match_batch call per step in each form (after an
    untimed warm-up), and the same images as 64 bm_match calls."""
    ws = synth.uneven_batch(64)
    ts = [torch.from_numpy(w_.image).to("cuda:0") for w_ in ws]
    n_ref = sum(w_.shape.n_ref for w_ in ws)
    flops = sum(2.0 * w_.shape.patch ** 2 * w_.shape.channels *
                pair_count(w_.shape.height, w_.shape.width, w_.shape.patch, w_.shape.stride,
                           w_.shape.window) for w_ in ws)
    stream = torch.cuda.current_stream()
    res = {"images": len(ws), "n_ref": n_ref, "algorithmic_flops": flops, "forms": {}}
    for prec in ["fp32", "bf16x4", "fp16x3"]:
        plans = [bm.cached_plan(bm.make_desc(w_.shape.height, w_.shape.width, w_.shape.channels,
                                             w_.shape.patch, w_.shape.stride, w_.shape.window,
                                             w_.shape.k, prec)) for w_ in ws]
        idxs = [torch.empty((p.n_ref, 16), dtype=torch.int32, device="cuda:0") for p in plans]
        dists = [torch.empty((p.n_ref, 16), dtype=torch.float32, device="cuda:0") for p in plans]
        wsb = torch.empty((bm.bm_batch_workspace(plans),), dtype=torch.uint8, device="cuda:0")

        def one_batch():
            bm.bm_match_batch(plans, ts, idxs, dists, wsb, stream)

        def per_image():
            for p, t, i, d in zip(plans, ts, idxs, dists):
                bm.bm_match(p, t, i, d, None, stream)

        entry = {}
        for name, fn, k in (("batch", one_batch, steps), ("per_image", per_image, 1)):
            warm(torch, fn, 1)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(k)]
            for a, b in ev:
                a.record(stream)
                fn()
                b.record(stream)
            torch.cuda.synchronize()
            ms = sum(a.elapsed_time(b) for a, b in ev) / k
            entry[name] = {"ms": ms, "value": n_ref / (ms / 1e3)}
        entry["roofline_frac"] = flops / (entry["batch"]["ms"] / 1e3) / 1e12 / PEAK_TFLOPS[prec]
        res["forms"][prec] = entry
    return res


def mfma_busy_from_profile(prec: str, workload: str):
    """Executed matrix-core utilisation of the cross-term kernel from the committed SQ
    counter summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"xcorr_{prec}_{workload}_sq_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != source_hash(prec):
        return None
    out = {}
    for k in ("mfma_busy_frac", "valu_busy_frac", "valu_per_tile", "mfma_per_tile"):
        try:
            out[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    return out or None


def bench_batch(args, bm, synth, torch):
    """The 64-image uneven workload: one bm_match_batch call per step."""
    import numpy as np
    ws = synth.uneven_batch(64, max_side=args.batch_max_side)
    ts = [torch.from_numpy(w.image).to("cuda:0") for w in ws]
    n_ref = sum(w.shape.n_ref for w in ws)
    flops = sum(2.0 * w.shape.patch ** 2 * w.shape.channels *
                pair_count(w.shape.height, w.shape.width, w.shape.patch, w.shape.stride,
                           w.shape.window) for w in ws)
    stream = torch.cuda.current_stream()
    forms = {}
    steps = max(3, min(args.steps, 20))
    for prec in ["fp32", "bf16x4", "fp16x3"]:
        plans = [bm.cached_plan(bm.make_desc(w.shape.height, w.shape.width, w.shape.channels,
                                             w.shape.patch, w.shape.stride, w.shape.window,
                                             w.shape.k, prec)) for w in ws]
        idxs = [torch.empty((p.n_ref, 16), dtype=torch.int32, device="cuda:0") for p in plans]
        dists = [torch.empty((p.n_ref, 16), dtype=torch.float32, device="cuda:0") for p in plans]
        wsb = torch.empty((bm.bm_batch_workspace(plans),), dtype=torch.uint8, device="cuda:0")

        def one_batch():
            bm.bm_match_batch(plans, ts, idxs, dists, wsb, stream)

        def per_image():
            for p, t, i, d in zip(plans, ts, idxs, dists):
                bm.bm_match(p, t, i, d, None, stream)

        res = {}
        for name, fn in (("batch", one_batch), ("per_image", per_image)):
            warm(torch, fn, 2)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(steps)]
            t0 = time.perf_counter()
            for a, b in ev:
                a.record(stream)
                fn()
                b.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ms = [a.elapsed_time(b) for a, b in ev]
            res[name] = {"value": n_ref * steps / wall, "ms_per_step": wall / steps * 1e3,
                         "p50_ms": quantile(ms, 0.5), "p99_ms": quantile(ms, 0.99)}
        forms[prec] = {"batch": res["batch"], "per_image": res["per_image"],
                       "configs": sorted({bm.bm_plan_config(p)[0] for p in plans})}
    prec = args.precision
    v = forms[prec]["batch"]["value"]
    step_s = forms[prec]["batch"]["ms_per_step"] / 1e3
    achieved = flops / step_s / 1e12
    out = {
        "metric": METRIC, "value": v, "unit": "ref-patches/s", "n_gpus": 1, "steps": steps,
        "warmup": 2, "ms_per_step": forms[prec]["batch"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": "uneven_batch64", "images": len(ws), "n_ref": n_ref,
                   "precision": prec, "seed0": 1000, "sides": [128, args.batch_max_side]},
        "latency_ms": {"p50": forms[prec]["batch"]["p50_ms"], "p99": forms[prec]["batch"]["p99_ms"]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[prec],
                     "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[prec], "traffic": None,
                     "kernel": "whole batch step (norms + persistent cross-term launches)",
                     "algorithmic_flops_per_launch": flops},
        "forms": forms,
        "plain_fp32": {"value": forms["fp32"]["per_image"]["value"],
                       "speedup": v / forms["fp32"]["per_image"]["value"]},
    }
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline_batch(ws, args.cpu_budget)
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(ws, budget_s):
    """FP64 oracle on 24 seeded references of each image in turn (bounded by budget_s)."""
    import numpy as np
    from oracle import bm_oracle as O
    rng = np.random.default_rng(5)
    done = 0
    t0 = time.perf_counter()
    for w in ws:
        refs = np.sort(rng.choice(w.shape.n_ref, size=min(24, w.shape.n_ref), replace=False))
        O.bm(w.image, w.shape.patch, w.shape.stride, w.shape.window, w.shape.k, refs=refs)
        done += len(refs)
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "ref-patches/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} references (24 seeded per image, images in order) of the "
                      f"64-image batch, numpy float64 brute force, {dt:.1f} s"}


def serve_sweep(bm, pool, prec, rates, seconds, n_clients):
    """Poisson request streams through the serving loop, one rate after another: per rate
    the achieved ref-patches/s and the p50/p99 request latency (submit to results on the
    host).  Requests replay `pool` cyclically; arrival gaps are Exp(1/QPS), seed QPS + 17."""
    import threading
    import numpy as np
    sweep = []
    for qps in rates:
        rng = np.random.default_rng(int(qps) + 17)
        n = max(8, int(qps * seconds))
        arrivals = np.cumsum(rng.exponential(1.0 / qps, size=n))
        arrivals -= arrivals[0]
        srv = bm.bm_server_create(32 << 30, max_inflight=64, max_queue=4096)
        outstanding = {}
        stats = []
        lock = threading.Lock()
        stop = threading.Event()

        def poller():
            while not stop.is_set() or outstanding:
                with lock:
                    items = list(outstanding.items())
                if not items:
                    time.sleep(0.0002)
                    continue
                for t, (w, d) in items:
                    st, s_ = bm.bm_poll(srv, t)
                    if st == bm.BM_OK:
                        with lock:
                            del outstanding[t]
                        stats.append((s_.total_s, s_.queue_s, s_.device_s, s_.n_ref, time.perf_counter()))
                time.sleep(0.0002)

        # warm: one request of each of the first four pool entries
        for w in pool[:4]:
            d = bm.make_desc(w.shape.height, w.shape.width, w.shape.channels, 8, 3, 39, 16, prec)
            t = bm.bm_submit(srv, d, w.image)
            while bm.bm_poll(srv, t)[0] != bm.BM_OK:
                time.sleep(0.001)
        th = threading.Thread(target=poller)
        th.start()
        t_start = time.perf_counter()
        counts = {"offered": 0, "rejected": 0}

        def client(c):
            # client c submits requests c, c + n_clients, ... at their arrival times
            for i in range(c, n, n_clients):
                w = pool[i % len(pool)]
                delay = t_start + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                d = bm.make_desc(w.shape.height, w.shape.width, w.shape.channels, 8, 3, 39, 16, prec)
                try:
                    t = bm.bm_submit(srv, d, w.image)
                    with lock:
                        outstanding[t] = (w, d)
                        counts["offered"] += w.shape.n_ref
                except bm.BMError as e:
                    if e.status != bm.BM_EBUSY:
                        raise
                    with lock:
                        counts["offered"] += w.shape.n_ref
                        counts["rejected"] += 1

        cl = [threading.Thread(target=client, args=(c,)) for c in range(n_clients)]
        for t_ in cl:
            t_.start()
        for t_ in cl:
            t_.join()
        offered, rejected = counts["offered"], counts["rejected"]
        t_submitted = time.perf_counter()
        stop.set()
        th.join()
        bm.bm_server_destroy(srv)
        t_end = max(s_[4] for s_ in stats) if stats else t_submitted
        done_refs = sum(s_[3] for s_ in stats)
        tot = sorted(s_[0] for s_ in stats)
        sweep.append({"qps": qps, "requests": n, "completed": len(stats), "rejected": rejected,
                      "offered_refs_per_s": offered / max(arrivals[-1], 1e-9),
                      "achieved_refs_per_s": done_refs / (t_end - t_start),
                      "p50_ms": 1e3 * quantile(tot, 0.5), "p99_ms": 1e3 * quantile(tot, 0.99),
                      "queue_p50_ms": 1e3 * quantile(sorted(s_[1] for s_ in stats), 0.5),
                      "device_p50_ms": 1e3 * quantile(sorted(s_[2] for s_ in stats), 0.5)})
        print(json.dumps({"serving_level": sweep[-1]}), file=sys.stderr, flush=True)
    return sweep


def bench_serving(args, bm, synth, torch):
    """Poisson request streams through the serving loop, one rate after another."""
    pool = [w for _, w in synth.serving_requests(16, 100.0)]
    prec = args.precision
    rates = [float(q) for q in args.qps.split(",") if q]
    sweep = serve_sweep(bm, pool, prec, rates, args.serve_seconds, args.clients)
    best = max(sweep, key=lambda r: r["achieved_refs_per_s"])
    # device capacity for this request mix: the pool as one resident batch, no host copies
    plans = [bm.cached_plan(bm.make_desc(w.shape.height, w.shape.width, w.shape.channels, 8, 3,
                                         39, 16, prec)) for w in pool]
    ts = [torch.from_numpy(w.image).to("cuda:0") for w in pool]
    idxs = [torch.empty((p.n_ref, 16), dtype=torch.int32, device="cuda:0") for p in plans]
    dists = [torch.empty((p.n_ref, 16), dtype=torch.float32, device="cuda:0") for p in plans]
    wsb = torch.empty((bm.bm_batch_workspace(plans),), dtype=torch.uint8, device="cuda:0")
    for _ in range(2):
        bm.bm_match_batch(plans, ts, idxs, dists, wsb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        bm.bm_match_batch(plans, ts, idxs, dists, wsb)
    torch.cuda.synchronize()
    capacity = 5 * sum(p.n_ref for p in plans) / (time.perf_counter() - t0)
    out = {
        "metric": METRIC, "value": best["achieved_refs_per_s"], "unit": "ref-patches/s",
        "n_gpus": 1, "steps": sum(r["completed"] for r in sweep), "warmup": 4,
        "ms_per_step": best["p50_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": "serving_poisson", "precision": prec, "pool": len(pool),
                   "clients": args.clients,
                   "sides": "log-uniform 256..2048", "channels": "1..4", "qps": rates},
        "latency_ms": {"p50": best["p50_ms"], "p99": best["p99_ms"]},
        "device_capacity_refs_per_s": capacity,
        "sweep": sweep,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
