#!/usr/bin/env python3
"""Throughput of the MI355X closed-curve alignment path.

Default workload: 65,536 independent pairs of closed curves with n = 1024
uniform arc-length nodes each, FP32, one call of align_batch per step (norms,
two forward FFTs, spectrum product, correlation FFT, argmax, FP64 re-scoring,
theta and e0 for every pair).  Inputs are seeded synthetic star curves; the
raw polygons are resampled to uniform arc length on the GPU before timing
(untimed) and stay resident in HBM.

Prints ONE JSON line (rank 0).  Other workloads: --config {pair,batch,allpairs,
ragged,bf16}; only the default line is the headline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
RESULT_BYTES = 32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default per workload, see DEFAULT_STEPS)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed warmup steps (default per workload, see DEFAULT_STEPS)")
    ap.add_argument("--config", default="batch",
                    choices=["batch", "pair", "allpairs", "ragged", "ragged_any", "bf16", "srv", "copy"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every step from Python instead of replaying a captured HIP graph")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target wall time of the CPU oracle sample")
    ap.add_argument("--settle-seconds", type=float, default=0.3,
                    help="untimed replays for this long before the warmup steps so the GPU clock "
                         "settles (reported as clock_settle; 0 = none)")
    args = ap.parse_args()
    steps, warmup = DEFAULT_STEPS[args.config]
    if args.steps is None:
        args.steps = steps
    if args.warmup is None:
        args.warmup = warmup
    return args


# Default (timed steps, warmup steps) per workload: the GPU's clock takes a
# few tens of milliseconds of load to settle (the batch workload's step time
# falls from ~0.42 ms in the first steps to ~0.35 ms), so the defaults give
# every workload >= 0.1 s of warmup and ~0.1-0.5 s of timed steps.
DEFAULT_STEPS = {"batch": (400, 300), "pair": (2000, 500), "allpairs": (40, 10), "ragged": (50, 15),
                 "ragged_any": (40, 10), "bf16": (200, 60), "srv": (300, 150), "copy": (200, 100)}


def sources_digest(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2501_17779_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


ALIGN_SOURCES = ["align.hip", "epilogue.hpp", "fft_engines.hpp", "dft_small.hpp", "common.hpp"]


def traffic_for(kernel_key: str, digest: str, per_launch_units: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    e = d.get(kernel_key)
    if not e or e.get("sources") != digest:
        return None
    return float(e["bytes_per_unit"]) * per_launch_units


def valu_issue_for(kernel_key: str, digest: str, per_launch_units: float, ms: float):
    """Fraction of the VALU issue cycles the kernel's wave instructions fill
    over a launch of ms milliseconds: VALU wave instructions per unit from the
    committed counter summary (taken on the current sources, else None) x 4
    cycles, over 1024 SIMDs at the nominal 2.4 GHz."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    e = d.get(kernel_key)
    if not e or e.get("sources") != digest or "valu_per_unit" not in e:
        return None
    return float(e["valu_per_unit"]) * per_launch_units * 4.0 / (ms * 1e-3 * 2.4e9 * 1024)


def graphed(fn, torch):
    """Capture one call of fn (its kernel launches) in a HIP graph; returns a
    replay function.  The first eager call builds the library's tables."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g.replay


# untimed replays before the warmup steps, per timed call (reported in the line)
SETTLE = {"seconds": 0.0, "replays": 0}
SETTLE_SECONDS = 0.0


def settle(fns, torch):
    """Replay the step for SETTLE_SECONDS of wall time before the warmup steps:
    the GPU clock takes tens of milliseconds of load to reach its steady
    value, and a handful of warmup steps is shorter than that."""
    if SETTLE_SECONDS <= 0:
        return
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < SETTLE_SECONDS:
        for _ in range(8):
            for f in fns:
                f()
        k += 8
        torch.cuda.synchronize()
    SETTLE["seconds"] += time.perf_counter() - t0
    SETTLE["replays"] += k


def time_steps(fn, steps, warmup, torch, graph=False):
    if graph:
        fn = graphed(fn, torch)
    settle([fn], torch)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    # two events bracket the timed steps; an event after every step (only for
    # BENCH_PER_STEP) adds its own cost to steps of a few microseconds
    per_step = bool(os.environ.get("BENCH_PER_STEP"))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1 if per_step else 2)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        fn()
        if per_step:
            ev[i + 1].record()
    ev[-1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if per_step:
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
        print("per-step ms:", " ".join(f"{x:.4f}" for x in per), file=sys.stderr, flush=True)
    return ev[0].elapsed_time(ev[-1]) / steps, wall


def time_parts(fns, steps, warmup, torch, graph=False):
    """Time a step made of several calls, with an event after each call, so
    that every call's average duration is measured inside the timed region.
    Each call is captured in a graph of its own when graph is set."""
    if graph:
        fns = [graphed(f, torch) for f in fns]
    settle(fns, torch)
    for _ in range(warmup):
        for f in fns:
            f()
    torch.cuda.synchronize()
    k = len(fns)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps * k + 1)]
    ev[0].record()
    for i in range(steps):
        for j, f in enumerate(fns):
            f()
            ev[i * k + j + 1].record()
    torch.cuda.synchronize()
    parts = [sum(ev[i * k + j].elapsed_time(ev[i * k + j + 1]) for i in range(steps)) / steps for j in range(k)]
    return ev[0].elapsed_time(ev[steps * k]) / steps, parts


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The paper's own timings of one alignment (Table 1; hardware, language and
# precision not stated): context for the measured numbers, not a target.
PAPER_TABLE1 = {"source": "paper Table 1 (one pair; hardware, language and precision not stated)",
                "n": [64, 128, 256, 512, 1024, 2048, 4096],
                "slow_s": [0.027, 0.06, 0.14, 0.31, 0.79, 2.2, 7.1],
                "fast_s": [0.005, 0.01, 0.02, 0.04, 0.07, 0.15, 0.30],
                "speedup_fast_vs_slow": [5.4, 6.9, 7.4, 7.5, 11.0, 15.0, 24.0]}


def full_batch_accuracy(z1, z2, res, nthreads=0):
    """Every pair of the batch against the FP64 oracle, which also supplies the
    CPU baseline: the slow method runs on the same FP32 nodes the GPU aligned
    and is read at the shift the GPU chose.  Returns (accuracy, cpu_baseline)."""
    import oracle
    t0 = time.perf_counter()
    r = oracle.check_batch_f32(z1, z2, res["shift"], nthreads=nthreads)
    dt = time.perf_counter() - t0
    B, n = z1.shape
    T0, T2, Ts = r["T"], r["T2"], r["T_at"]
    with np.errstate(divide="ignore", invalid="ignore"):
        gap = np.where(T0 > 0, (T0 - T2) / T0, 0.0)
        excess = np.where(T0 > 0, (T0 - Ts) / T0, 0.0)
    s0 = (n - r["m"]) % n
    near = gap < 1e-6
    mism = (~near) & (res["shift"] != s0)
    # the acceptance rule: the oracle's shift, or at a near-tie a shift within 1e-6 of its value
    outside = (res["shift"] != s0) & ((~near) | (excess > 1e-6))
    dth = np.abs(oracle.wrap_angle(res["theta"] - oracle.wrap_angle(-r["theta_paper_at"])))
    de = np.abs(res["e0"] - r["E_at"]) / np.maximum(r["E_at"], 1e-300)
    acc = {"pairs": int(B), "theta_err_max": float(dth.max()), "theta_err_mean": float(dth.mean()),
           "e0_rel_err_max": float(de.max()), "e0_rel_err_mean": float(de.mean()),
           "shift_mismatch_outside_near_ties": int(mism.sum()), "near_ties": int(near.sum()),
           "outside_acceptance_rule": int(outside.sum()),
           "shift_equal_to_oracle": int((res["shift"] == s0).sum()),
           "shift_rel_excess_max": float(excess.max())}
    base = {"value": B / dt, "unit": "pairs/s", "cores": int(r["threads"]), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"all {B} pairs of the workload (n={n}) on the GPU-resampled nodes, FP64 slow method "
                      f"(+ one energy sum per pair at the GPU's shift), {dt:.1f} s wall on {r['threads']} threads"}
    return acc, base


def cpu_baseline_batch(get_pairs, total, n, seconds, what="first {k} of the workload's pairs"):
    """The FP64 oracle (slow method, OpenMP over pairs) on a bounded sample of
    the workload's pairs: the sample grows until one run takes `seconds` (or
    covers all `total` pairs), and that run is reported.  get_pairs(k) returns
    the first k pairs as float32 (k, n, 2) arrays; the oracle's cost does not
    depend on the node values."""
    import oracle

    def zs(k):
        a, b = get_pairs(k)
        return ((a[..., 0] + 1j * a[..., 1]).astype(np.complex64),
                (b[..., 0] + 1j * b[..., 1]).astype(np.complex64))

    k = min(64, total)
    while True:
        z1, z2 = zs(k)
        t0 = time.perf_counter()
        _, _, _, _, used = oracle.align_batch_f32(z1, z2)
        dt = time.perf_counter() - t0
        if dt >= seconds or k >= total:
            break
        k = int(min(total, max(2 * k, 1.1 * k * seconds / max(dt, 1e-6))))
    return {"value": k / dt, "unit": "pairs/s", "cores": int(used), "kind": "oracle", "cpu_model": cpu_model(),
            "sample": what.format(k=k) + f" (n={n}), FP64 slow method, {dt:.1f} s wall on {used} threads"}


def bench_batch(args, torch, ca):
    from synth import curves
    B, n = 65536, 1024
    dev = torch.device("cuda:0")
    r1, r2 = curves.batch_pairs_torch(17780, B, n, dev)
    raw = torch.view_as_complex(torch.cat([r1, r2]).reshape(-1, 2)).contiguous()
    roff = torch.arange(0, 2 * B + 1, dtype=torch.int64, device=dev) * n
    nodes, _, flags = ca.resample_arclength(raw, roff, roff)
    z1 = nodes[: B * n].view(B, n)
    z2 = nodes[B * n:].view(B, n)
    out = ca.empty_results(B, dev)
    torch.cuda.synchronize()
    assert int((flags != 0).sum().item()) == 0
    ms, wall = time_steps(lambda: ca.align_batch(z1, z2, out=out), args.steps, args.warmup, torch,
                          graph=not args.no_graph)
    algo_bytes = B * (2 * n * 8 + RESULT_BYTES)
    achieved = algo_bytes / (ms * 1e-3) / 1e9
    traffic = traffic_for("k_align_team_1024", sources_digest(ALIGN_SOURCES), B)
    line = {
        "metric": "curve-pair alignments/sec at N=1024, FP32 vs split-BF16, err vs FP64 oracle",
        "value": B / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch of 65536 curve pairs, n=1024 nodes, FP32, top-2 FP64 re-scoring",
                   "pairs": B, "n": n, "rescore": "top2"},
        "roofline": {"bound": "hbm", "kernel": "k_align_team<1024>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "valu_issue": valu_issue_for("k_align_team_1024", sources_digest(ALIGN_SOURCES), B, ms)},
    }
    # the same inputs through the split-BF16 MFMA path (the metric's second half)
    res32 = ca.to_numpy(out)
    out16 = ca.empty_results(B, dev)
    ms16, _ = time_steps(lambda: ca.align_batch(z1, z2, precision="split_bf16", out=out16), args.steps,
                         args.warmup, torch, graph=not args.no_graph)
    mfma_flops = B * MFMA_FLOPS_PER_PAIR_1024
    line["split_bf16"] = {
        "value": B / (ms16 * 1e-3), "unit": "pairs/s", "ms_per_step": ms16, "speedup_vs_fp32": ms / ms16,
        "dtype": "bf16x3 (fp32 accumulate, fp64 shift search and e0)",
        "roofline": {"bound": "mfma", "kernel": "k_align_bf16_1k",
                     "achieved": mfma_flops / (ms16 * 1e-3) / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": mfma_flops / (ms16 * 1e-3) / 1e12 / 2500.0,
                     "hbm_frac": algo_bytes / (ms16 * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    if not args.no_cpu_baseline:
        z1h, z2h = z1.cpu().numpy(), z2.cpu().numpy()
        acc, base = full_batch_accuracy(z1h, z2h, res32)
        line["cpu_baseline"] = base
        line["accuracy"] = {"fp32": acc}
        acc16, _ = full_batch_accuracy(z1h, z2h, ca.to_numpy(out16))
        line["accuracy"]["split_bf16"] = acc16
    line["paper_context"] = PAPER_TABLE1
    return line


# MFMA work of the n = 1024 split-BF16 path per pair: three transforms x two
# 32-point stages x (4 K-blocks x 2 output blocks x 3 split products) of
# v_mfma_f32_32x32x16_bf16 (32 x 32 x 16 multiply-adds = 32,768 flops each).
MFMA_FLOPS_PER_PAIR_1024 = 3 * 2 * 24 * 32 * 32 * 16 * 2


HEADLINE_METRIC = "curve-pair alignments/sec at N=1024, FP32 vs split-BF16, err vs FP64 oracle"
# FP32 and FP64 vector issue peaks without packed FP32 instructions (not used
# by this build): 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
VALU_FP32_PEAK_TFLOPS = 78.6


def base_line(args, value, unit, ms, dtype, config, higher=True):
    return {"metric": HEADLINE_METRIC if config.get("headline") else config["workload"],
            "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None,
            "dtype": dtype, "data": "synthetic",
            "config": {k: v for k, v in config.items() if k != "headline"}}


def bench_pair(args, torch, ca):
    """One pair, n = 256, FP64 block engine: latency of one align_pair call."""
    from synth import curves
    dev = torch.device("cuda:0")
    r1, r2 = curves.batch_pairs_torch(17779, 1, 256, dev, kmin=8, kmax=8, sigma_max=1e-3)
    raw = torch.view_as_complex(torch.cat([r1, r2]).reshape(-1, 2)).contiguous()
    off = torch.arange(0, 3, dtype=torch.int64, device=dev) * 256
    nodes, _, _ = ca.resample_arclength(raw, off, off)
    z = nodes.to(torch.complex128)
    z1, z2 = z[:256].contiguous(), z[256:].contiguous()
    out = ca.empty_results(1, dev)
    steps = args.steps
    ms, _ = time_steps(lambda: ca.align_pair(z1, z2, precision="fp64", out=out), steps, args.warmup, torch)
    line = base_line(args, 1e3 / ms, "pairs/s", ms, "f64",
                     {"workload": "single curve pair, n=256 nodes, FP64 (latency of one call)",
                      "pairs": 1, "n": 256})
    line["us_per_call"] = ms * 1e3
    msg, _ = time_steps(lambda: ca.align_pair(z1, z2, precision="fp64", out=out), steps, args.warmup, torch,
                        graph=True)
    line["us_per_call_graph_replay"] = msg * 1e3
    return line


def bench_allpairs(args, torch, ca):
    """All 8,386,560 pairs of a 4096-curve gallery at n = 512, FP32."""
    from synth import curves
    M, n = 4096, 512
    dev = torch.device("cuda:0")
    raw = torch.view_as_complex(curves.gallery_torch(17781, M, 2048, dev).reshape(-1, 2)).contiguous()
    roff = torch.arange(0, M + 1, dtype=torch.int64, device=dev) * 2048
    ooff = torch.arange(0, M + 1, dtype=torch.int64, device=dev) * n
    g, _, _ = ca.resample_arclength(raw, roff, ooff)
    g = g.view(M, n)
    P = M * (M - 1) // 2
    out = ca.empty_results(P, dev)
    ms, _ = time_steps(lambda: ca.align_all_pairs(g, out=out), args.steps, args.warmup, torch,
                       graph=not args.no_graph)
    flops = P * (5 * n * 9 + 9 * n)       # correlation FFT + product + |C|^2, per pair
    achieved = flops / (ms * 1e-3) / 1e12
    line = base_line(args, P / (ms * 1e-3), "pairs/s", ms, "f32",
                     {"workload": "all pairs of a 4096-curve gallery, n=512 nodes, FP32", "curves": M,
                      "pairs": P, "n": n})
    traffic = traffic_for("k_allpairs_512", sources_digest(ALIGN_SOURCES), P)
    line["roofline"] = {"bound": "alu", "kernel": "k_allpairs<512>", "achieved": achieved,
                        "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / VALU_FP32_PEAK_TFLOPS, "traffic": traffic,
                        "valu_issue": valu_issue_for("k_allpairs_512", sources_digest(ALIGN_SOURCES), P, ms)}
    if not args.no_cpu_baseline:
        gh = g.cpu().numpy()
        ii, jj = np.triu_indices(M, 1)

        def pairs(k):
            return (np.stack([gh[ii[:k]].real, gh[ii[:k]].imag], -1),
                    np.stack([gh[jj[:k]].real, gh[jj[:k]].imag], -1))

        line["cpu_baseline"] = cpu_baseline_batch(pairs, P, n, args.cpu_seconds,
                                                  "first {k} pairs of the gallery in upper-triangle order")
    return line


def bench_ragged(args, torch, ca, snap=True):
    """100,000 pairs of raw polygons, n log-uniform in [64, 4096] (7-smooth,
    or any integer with snap=False), 1.2-5x more raw vertices than n: GPU
    resampling + ragged alignment per step."""
    from synth import curves
    B = 100000
    dev = torch.device("cuda:0")
    d = curves.ragged_pairs_torch(17782, B, dev, snap=snap)
    raw = torch.cat([d["raw1"], d["raw2"]])
    roff = torch.cat([d["off1"], d["off2"][1:] + d["off1"][-1]])
    n = d["n"].long()
    ooff = torch.zeros(2 * B + 1, dtype=torch.int64, device=dev)
    ooff[1:] = torch.cumsum(torch.cat([n, n]), 0)
    total = int(ooff[-1].item())
    nodes = torch.empty(total, dtype=torch.complex64, device=dev)
    off = ooff[: B + 1].contiguous()
    half = int(off[-1].item())
    out = ca.empty_results(B, dev)

    def resample(stream=None):
        ca.resample_arclength(raw, roff, ooff, out=nodes, with_norms=False, with_flags=False, stream=stream)

    def align(stream=None):
        ca.align_batch(nodes[:half], nodes[half:], offsets=off, out=out, stream=stream)

    # each call in a graph of its own, an event after each: the parts' times
    ms_parts, (ms_rs, ms_al) = time_parts([resample, align], args.steps, args.warmup, torch,
                                          graph=not args.no_graph)
    # the step: both calls recorded in one library-owned graph, one launch per step
    if args.no_graph:
        ms, _ = time_steps(lambda: (resample(), align()), args.steps, args.warmup, torch)
    else:
        lg = ca.capture(lambda st: (resample(st), align(st)))
        ms, _ = time_steps(lg.launch, args.steps, args.warmup, torch)
    # dominant kernel: the resampler (reads every raw vertex and both offset
    # arrays, writes every node)
    algo = raw.numel() * 8 + total * 8 + 2 * (2 * B + 1) * 8
    achieved = algo / (ms_rs * 1e-3) / 1e9
    wl = ("100000 ragged pairs of raw polygons, n in [64,4096], GPU resampling + alignment" if snap else
          "100000 ragged pairs of raw polygons, any integer n in [64,4096] (zero-padded transforms for n "
          "with a prime factor above 7), GPU resampling + alignment")
    line = base_line(args, B / (ms * 1e-3), "pairs/s", ms, "f32",
                     {"workload": wl, "pairs": B, "raw_vertices": int(raw.numel()), "nodes": total,
                      "n_7smooth": bool(snap)})
    line["parts_ms"] = {"resample_arclength": ms_rs, "align_batch_ragged": ms_al,
                        "note": "each call in its own graph with events between (sum %.3f ms); ms_per_step "
                                "is one library graph (ca_graph_begin/end) of both calls" % ms_parts}
    traffic = traffic_for("k_resample_fast", sources_digest(["resample.hip", "common.hpp"]), 1.0)
    line["roofline"] = {"bound": "hbm", "kernel": "k_resample_fast", "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": traffic,
                        "valu_issue": valu_issue_for("k_resample_fast", sources_digest(["resample.hip", "common.hpp"]),
                                                     1.0, ms_rs) if snap else None}
    return line


def accuracy_sample(torch, ca, raw1, raw2, n, precisions, k=256):
    """Accuracy against the FP64 oracle on k pairs of the workload: the raw
    polygons are resampled by the oracle, aligned on the GPU with each
    precision and by the oracle, and compared (max/mean theta and e0 error,
    shift mismatches outside near-ties, and the largest relative shortfall
    (T(s0) - T(shift)) / T(s0) of the chosen shift's |C| below the oracle's
    maximum: at a near-tie any shift within 1e-6 is accepted)."""
    import oracle
    from oracle import resample_ref as rr
    z1 = np.stack([rr.resample(raw1[i].astype(np.float64), n)[0] for i in range(k)]).astype(np.complex64)
    z2 = np.stack([rr.resample(raw2[i].astype(np.float64), n)[0] for i in range(k)]).astype(np.complex64)
    orc = []
    for i in range(k):
        T, th, m, thp = oracle.per_shift_arrays(z1[i], z2[i])
        orc.append((T, th, m, thp))
    out = {}
    for prec in precisions:
        res = ca.to_numpy(ca.align_batch(torch.from_numpy(z1).cuda(), torch.from_numpy(z2).cuda(),
                                         precision=prec))
        dth, de, mism, near, excess = [], [], 0, 0, 0.0
        for i in range(k):
            T, th, m, thp = orc[i]
            s0 = int(np.argmax(T))
            T2 = np.max(np.delete(T, s0))
            s = int(res["shift"][i])
            excess = max(excess, float((T[s0] - T[s]) / T[s0]))
            if (T[s0] - T2) / T[s0] < 1e-6:
                near += 1
            elif s != s0:
                mism += 1
            dth.append(abs(float(oracle.wrap_angle(res["theta"][i] - th[s]))))
            E = oracle.energy(z1[i], z2[i], int(m[s]), float(thp[s]))
            de.append(abs(res["e0"][i] - E) / max(E, 1e-300))
        out[prec] = {"pairs": k, "theta_err_max": max(dth), "theta_err_mean": float(np.mean(dth)),
                     "e0_rel_err_max": max(de), "e0_rel_err_mean": float(np.mean(de)),
                     "shift_mismatch_outside_near_ties": mism, "near_ties": near,
                     "shift_rel_excess_max": excess}
    return out


def bench_small_batch(args, torch, ca):
    """1,048,576 pairs at n = 128: split-BF16 MFMA path, with the FP32 FFT path
    timed on the same inputs."""
    from synth import curves
    B, n = 1 << 20, 128
    dev = torch.device("cuda:0")
    r1, r2 = curves.batch_pairs_torch(17783, B, n, dev, kmin=8, kmax=8, sigma_max=1e-3)
    raw = torch.view_as_complex(torch.cat([r1, r2]).reshape(-1, 2)).contiguous()
    roff = torch.arange(0, 2 * B + 1, dtype=torch.int64, device=dev) * n
    nodes, _, _ = ca.resample_arclength(raw, roff, roff)
    z1, z2 = nodes[: B * n].view(B, n), nodes[B * n:].view(B, n)
    out = ca.empty_results(B, dev)
    ms16, _ = time_steps(lambda: ca.align_batch(z1, z2, precision="split_bf16", out=out), args.steps,
                         args.warmup, torch, graph=not args.no_graph)
    ms32, _ = time_steps(lambda: ca.align_batch(z1, z2, out=out), args.steps, args.warmup, torch,
                         graph=not args.no_graph)
    flops = B * 3 * 3 * (2 * 32 * 32 * 8 + 2 * 16 * 16 * 16)   # split products x transforms x stages
    achieved = flops / (ms16 * 1e-3) / 1e12
    line = base_line(args, B / (ms16 * 1e-3), "pairs/s", ms16, "bf16x3 (fp32 accumulate)",
                     {"workload": "batch of 1048576 curve pairs, n=128 nodes, split-BF16 MFMA DFT vs FP32 FFT",
                      "pairs": B, "n": n})
    line["fp32_same_inputs"] = {"value": B / (ms32 * 1e-3), "ms_per_step": ms32,
                                "hbm_frac": B * (2 * n * 8 + RESULT_BYTES) / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS}
    line["speedup_vs_fp32"] = ms32 / ms16
    traffic = traffic_for("k_align_bf16", sources_digest(["bf16.hip"] + ALIGN_SOURCES[1:]), B)
    line["roofline"] = {"bound": "mfma", "kernel": "k_align_bf16", "achieved": achieved, "peak": 2500.0,
                        "unit": "TFLOP/s", "frac": achieved / 2500.0, "traffic": traffic,
                        "valu_issue": valu_issue_for("k_align_bf16", sources_digest(["bf16.hip"] + ALIGN_SOURCES[1:]),
                                                     B, ms16)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(lambda k: (r1[:k].cpu().numpy(), r2[:k].cpu().numpy()), B, n,
                                                  args.cpu_seconds)
        line["accuracy"] = accuracy_sample(torch, ca, r1[:256].cpu().numpy(), r2[:256].cpu().numpy(), n,
                                           ["fp32", "split_bf16"])
    return line


def bench_srv(args, torch, ca):
    """The (t0, R) step of the elastic solver on SRV functions (section 3) at
    the batch workload's size: SRV transform of both curves of 65,536 pairs
    (n = 1024), then the alignment of (q2, q1), every step."""
    from synth import curves
    B, n = 65536, 1024
    dev = torch.device("cuda:0")
    r1, r2 = curves.batch_pairs_torch(17780, B, n, dev)
    raw = torch.view_as_complex(torch.cat([r1, r2]).reshape(-1, 2)).contiguous()
    roff = torch.arange(0, 2 * B + 1, dtype=torch.int64, device=dev) * n
    nodes, _, _ = ca.resample_arclength(raw, roff, roff)
    nodes = nodes.view(2 * B, n)
    q = torch.empty_like(nodes)
    out = ca.empty_results(B, dev)

    def srv():
        ca.srv_transform(nodes, out=q)

    def align():
        ca.align_batch(q[B:], q[:B], out=out)

    ms, (ms_srv, ms_al) = time_parts([srv, align], args.steps, args.warmup, torch, graph=not args.no_graph)
    line = base_line(args, B / (ms * 1e-3), "pairs/s", ms, "f32",
                     {"workload": "SRV (t0, R) step: SRV transform of 65536 curve pairs, n=1024, then "
                                  "alignment of (q2, q1), FP32, top-2 FP64 re-scoring", "pairs": B, "n": n})
    line["parts_ms"] = {"srv_transform": ms_srv, "align_batch": ms_al}
    algo = B * (2 * n * 8 + RESULT_BYTES)
    achieved = algo / (ms_al * 1e-3) / 1e9
    line["roofline"] = {"bound": "hbm", "kernel": "k_align_team<1024>", "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": traffic_for("k_align_team_1024", sources_digest(ALIGN_SOURCES), B),
                        "valu_issue": valu_issue_for("k_align_team_1024", sources_digest(ALIGN_SOURCES), B, ms_al)}
    srv_gbs = 2 * B * n * 16 / (ms_srv * 1e-3) / 1e9
    line["srv_roofline"] = {"bound": "hbm", "kernel": "k_srv", "achieved": srv_gbs, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": srv_gbs / HBM_PEAK_GBS,
                            "traffic": traffic_for("k_srv", sources_digest(["srv.hip", "common.hpp"]), 2 * B * n)}
    return line


def bench_copy(args, torch, ca):
    """A plain device-to-device copy of 1 GiB: the reference reading for the
    rocprofv3 FETCH_SIZE / WRITE_SIZE counters (bytes moved are known)."""
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    ms, _ = time_steps(lambda: dst.copy_(src), args.steps, args.warmup, torch)
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    return {"metric": "device copy bandwidth", "value": gbs, "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "copy of 1 GiB (read 1 GiB + write 1 GiB)", "bytes": nbytes}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus "
              f"{args.gpus}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2501_17779_amd as ca
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    ctx = ca.default_context(0)
    global SETTLE_SECONDS
    SETTLE_SECONDS = args.settle_seconds
    fn = {"batch": bench_batch, "copy": bench_copy, "pair": bench_pair, "allpairs": bench_allpairs,
          "ragged": bench_ragged, "ragged_any": lambda a, t, c: bench_ragged(a, t, c, snap=False),
          "bf16": bench_small_batch, "srv": bench_srv}[args.config]
    line = fn(args, torch, ca)
    # launch choices in force: the tuning cache default_context loaded (if any)
    src = os.environ.get("CURVEALIGN_TUNE_FILE", ca.TUNE_CACHE)
    line["clock_settle"] = {"seconds": round(SETTLE["seconds"], 3), "replays": SETTLE["replays"],
                            "note": "untimed replays before the warmup steps (GPU clock ramp)"}
    line["tuning"] = {"cache": os.path.relpath(src, ROOT) if src and os.path.exists(src) else None,
                      "entries_applied": getattr(ctx, "tune_applied", 0)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
