#!/usr/bin/env python3
"""Benchmark of the AB-join hot path on one MI355X.

One step = one full ``ab_join`` call (window statistics, pair loop, row
reduction, FP64 winner re-check) of the dictionary inference workload:
an ECG-like query of 131,072 samples against a dictionary of 16 segments x
2,000 samples, m = 256 (windows that cross a segment break are masked).
Inputs are resident in device memory before the timed region.

Prints ONE JSON line.  ``value`` = valid (query window, dictionary window)
pairs per second over the timed steps.  ``roofline`` is for the pair-loop
kernel, timed with HIP events that the library records on the stream it
launches the kernel on.  ``cpu_baseline`` is the FP64 oracle on a bounded
sample of query rows of the same workload, on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "ecg131k_dict16x2000_m256"
METRIC = "AB-join subsequence-pair distances/s vs plain FP32 at stated error; p99 latency"
VALU_PEAK = 256 * 4 * 16 * 2.4e9  # lane-ops/s: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
OPS_PER_PAIR = 4  # 2 FMA (covariance step) + 1 MUL (normalise) + 1 compare (running max)


def profiled_traffic(kernel_source: str, summary: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None
    when the kernel source has changed since the counters were taken."""
    import hashlib

    try:
        fields = dict(l.split(": ", 1) for l in open(summary).read().splitlines() if ": " in l)
        sha = hashlib.sha256(open(kernel_source, "rb").read()).hexdigest()
        if fields.get("kernel_source_sha256") == sha:
            return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        pass
    return None


def valid_windows(bounds, m):
    b = np.asarray(bounds)
    return int(sum(max(0, int(b[s + 1] - b[s]) - m + 1) for s in range(len(b) - 1)))


def cpu_baseline(w, P_gpu, I_gpu, target_s: float, threads: int):
    """Time the FP64 oracle on a bounded row sample; also report the GPU error there."""
    import oracle

    q, d, b, m = w["query"], w["dict"], w["bounds"], w["m"]
    W = len(q) - m + 1
    V = valid_windows(b, m)
    rng = np.random.default_rng(12345)
    cal = np.sort(rng.choice(W, 64, replace=False))
    t0 = time.perf_counter()
    oracle.ab_join(q, d, b, m, rows=cal, threads=threads)
    t_cal = time.perf_counter() - t0
    nrows = int(np.clip(64 * target_s / max(t_cal, 1e-3), 64, W))
    rows = np.sort(rng.choice(W, nrows, replace=False))
    t0 = time.perf_counter()
    Po, Io = oracle.ab_join(q, d, b, m, rows=rows, threads=threads)
    dt = time.perf_counter() - t0
    err = np.abs(P_gpu[rows].astype(np.float64) - Po)
    return (
        {"value": nrows * V / dt, "unit": "pair-distances/s", "cores": threads, "kind": "oracle",
         "sample": f"{nrows} random query rows x {V} dictionary windows of the same workload, "
                   f"{dt:.1f} s wall, FP64 brute force, OpenMP {threads} threads"},
        {"rows": nrows, "max_abs": float(err.max()), "mean_abs": float(err.mean()),
         "index_match": float(np.mean(I_gpu[rows] == Io))},
    )


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tier", default="fp32", choices=["fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the timed steps, run one device-to-device copy of this many bytes "
                         "(reference dispatch for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2112_12965_amd import abjoin, synth

    w = synth.WORKLOADS[WORKLOAD]()
    m, bounds = w["m"], w["bounds"]
    q = torch.from_numpy(w["query"]).cuda()
    d = torch.from_numpy(w["dict"]).cuda()
    WA = len(w["query"]) - m + 1
    V = valid_windows(bounds, m)
    pairs = WA * V
    P = torch.empty(WA, dtype=torch.float32, device="cuda")
    I = torch.empty(WA, dtype=torch.int64, device="cuda")
    L = abjoin.lib()

    for _ in range(args.warmup):
        abjoin.ab_join(q, d, bounds, m, tier=args.tier, out=(P, I))
    torch.cuda.synchronize()
    L.abj_profile_enable(1)
    abjoin.lib().abj_profile_read(None, None, None)  # clear
    t0 = time.perf_counter()
    for _ in range(args.steps):
        abjoin.ab_join(q, d, bounds, m, tier=args.tier, out=(P, I))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    import ctypes

    kms, nl, kp = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
    L.abj_profile_read(ctypes.byref(kms), ctypes.byref(nl), ctypes.byref(kp))
    L.abj_profile_enable(0)
    if args.copy_bytes > 0:
        src = torch.empty(args.copy_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    kernel_ms = kms.value / max(nl.value, 1)
    kernel_pairs = kp.value / max(nl.value, 1)
    achieved = OPS_PER_PAIR * kernel_pairs / (kernel_ms * 1e-3)

    out = {
        "metric": METRIC,
        "value": pairs * args.steps / dt,
        "unit": "pair-distances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "query_samples": len(w["query"]), "dict_segments": len(bounds) - 1,
                   "segment_samples": int(bounds[1] - bounds[0]), "m": m, "tier": args.tier,
                   "pairs_per_step": pairs},
        "roofline": {"bound": "alu", "kernel": "k_join_fp32", "achieved": achieved / 1e12,
                     "peak": VALU_PEAK / 1e12, "unit": "TOP/s (VALU lane-ops)",
                     "frac": achieved / VALU_PEAK, "ops_per_pair": OPS_PER_PAIR,
                     "kernel_ms": kernel_ms,
                     "traffic": profiled_traffic(
                         os.path.join(ROOT, "paper_2112_12965_amd", "csrc", "join_fp32.hip"),
                         os.path.join(ROOT, "profiles", "k_join_fp32_ecg131k_dict16x2000_m256_hbm_counters.md"))},
    }
    if not args.no_cpu:
        Ph, Ih = P.cpu().numpy(), I.cpu().numpy()
        threads = min(16, os.cpu_count() or 1)
        cb, err = cpu_baseline(w, Ph, Ih, args.cpu_seconds, threads)
        out["cpu_baseline"] = cb
        out["error_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
