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
# issue ceiling of FMA-class VALU instructions (FP32 FMA and multiply, FP64 FMA)
# without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9
METRIC = "AB-join subsequence-pair distances/s vs plain FP32 at stated error; p99 latency"
# FP32 vector peak of MI355X: 256 CUs x 128 FP32 lanes x 2 flops (FMA) x 2.4 GHz
FP32_PEAK = 157.3e12
# per pair: 2 FMA (diagonal covariance step) + 1 multiply (column weight) + 1 max (running best)
FLOPS_PER_PAIR = 2 * 2 + 1 + 1


def profiled_field(kernel_source: str, summary: str, field: str):
    """A figure from a committed rocprofv3 counter summary, or None when the
    kernel source has changed since the counters were taken."""
    import hashlib

    try:
        fields = dict(l.split(": ", 1) for l in open(summary).read().splitlines() if ": " in l)
        sha = hashlib.sha256(open(kernel_source, "rb").read()).hexdigest()
        if fields.get("kernel_source_sha256") == sha:
            return float(fields[field])
    except (OSError, KeyError, ValueError):
        pass
    return None


def valid_windows(bounds, m):
    b = np.asarray(bounds)
    return int(sum(max(0, int(b[s + 1] - b[s]) - m + 1) for s in range(len(b) - 1)))


def cpu_baseline(w, results, target_s: float, threads: int):
    """Time the FP64 oracle on a bounded row sample; report each GPU tier's error there.

    ``results``: {tier: (P, I)} host arrays of the full GPU result.  The oracle
    is timed on a 64-row call first, then on as many rows as fit in about
    ``target_s`` seconds."""
    import oracle

    q, d, b, m = w["query"], w["dict"], w["bounds"], w["m"]
    W = len(q) - m + 1
    V = valid_windows(b, m)
    rng = np.random.default_rng(12345)
    t0 = time.perf_counter()
    oracle.ab_join(q, d, b, m, rows=np.sort(rng.choice(W, 64, replace=False)), threads=threads)
    t64 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.ab_join(q, d, b, m, rows=np.sort(rng.choice(W, 256, replace=False)), threads=threads)
    t256 = time.perf_counter() - t0
    per_row = max((t256 - t64) / 192.0, 1e-6)  # the call's fixed cost cancels
    nrows = int(np.clip(target_s / per_row, 256, W))
    rows = np.sort(rng.choice(W, nrows, replace=False))
    t0 = time.perf_counter()
    Po, Io, P2o = oracle.ab_join(q, d, b, m, rows=rows, threads=threads, second=True)
    dt = time.perf_counter() - t0
    errs = {}
    for tier, (P, I) in results.items():
        err = np.abs(P[rows].astype(np.float64) - Po)
        clear = (P2o - Po) > 1e-3
        errs[tier] = {"rows": nrows, "max_abs": float(err.max()), "mean_abs": float(err.mean()),
                      "index_match_clear_rows": float(np.mean(I[rows][clear] == Io[clear]))}
    return (
        {"value": nrows * V / dt, "unit": "pair-distances/s", "cores": threads, "kind": "oracle",
         "sample": f"{nrows} random query rows x {V} dictionary windows of the same workload, "
                   f"{dt:.1f} s wall, FP64 brute force, OpenMP {threads} threads"},
        errs,
    )


def short_windows(abjoin, synth, ms=(16, 32, 64), n=262144, rows=192):
    """Tiers against short windows: whole-step pairs/s of every tier on two
    n-sample random walks per m.  Returns the record and, for the CPU leg's
    error check, each tier's result on `rows` random query rows."""
    import torch

    rng = synth.rng_for(7, 0)
    a_h, b_h = synth.random_walk(n, rng), synth.random_walk(n, rng)
    a, b = torch.from_numpy(a_h).cuda(), torch.from_numpy(b_h).cuda()
    out = {"workload": f"random walks {n} x {n}", "m": {}}
    samples = {}
    for m in ms:
        W = n - m + 1
        rec = {}
        sample = np.sort(np.random.default_rng(100 + m).choice(W, rows, replace=False))
        got = {}
        for tier in ("fp32", "bf16", "fp16"):
            P = torch.empty(W, dtype=torch.float32, device="cuda")
            I = torch.empty(W, dtype=torch.int64, device="cuda")
            dt = time_tier(abjoin, a, b, [0, n], m, tier, 5, 2, P, I)
            rec[tier] = {"pairs_per_s": W * W / dt, "ms_per_step": dt * 1e3}
            got[tier] = (P.cpu().numpy().astype(np.float64)[sample], I.cpu().numpy()[sample])
        for tier in ("bf16", "fp16"):
            rec[tier]["vs_fp32"] = rec[tier]["pairs_per_s"] / rec["fp32"]["pairs_per_s"]
        out["m"][str(m)] = rec
        samples[m] = (sample, got)
    return out, (a_h, b_h, samples)


def short_window_errors(record, data, threads):
    """Each tier's error on the sampled rows against the FP64 oracle (CPU leg)."""
    import oracle

    a_h, b_h, samples = data
    n = len(a_h)
    for m, (rows, got) in samples.items():
        Po, Io, P2o = oracle.ab_join(a_h, b_h, [0, n], m, rows=rows, threads=threads, second=True)
        clear = (P2o - Po) > 1e-3
        for tier, (Pg, Ig) in got.items():
            r = record["m"][str(m)][tier]
            r["rows_checked"] = int(len(rows))
            r["max_abs_err"] = float(np.abs(Pg - Po).max())
            r["index_match_clear_rows"] = float(np.mean(Ig[clear] == Io[clear])) if clear.any() else 1.0


def pipeline(abjoin, synth, n=262144, n_series=8, m=256, space_saving=0.9, K=50):
    """The whole method at the size of the database workload: the learning
    phase (Alg. 1) on each of n_series ECG-like database series, their
    dictionaries concatenated into one, each of n_series held-out series (50
    planted anomalous beats) joined against it (Alg. 2), and its exact top-K
    discords against the whole database from that join (Lemmas 1-2).  e_max is
    the largest of the per-series values, an upper bound for the concatenated
    dictionary.  Reports the time of each phase and how many planted beats the
    discords hit (a discord within one beat, 260 samples, of a planted start)."""
    import torch

    db = [synth.ecg_like(n, synth.rng_for(11, k)) for k in range(n_series)]
    held = [synth.ecg_like(n, synth.rng_for(12, k), n_anomalies=50, return_anomalies=True) for k in range(n_series)]
    db_dev = [torch.from_numpy(x).cuda() for x in db]
    held_dev = [torch.from_numpy(x).cuda() for x, _ in held]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    learned = [abjoin.dict_build(x, m, stop="space_saving", value=space_saving) for x in db_dev]
    torch.cuda.synchronize()
    t_learn = time.perf_counter() - t0
    D = torch.cat([g["dictionary"] for g in learned])
    dbounds = [0]
    for g in learned:
        dbounds += [dbounds[-1] + int(b) for b in g["bounds"][1:]]
    e_max = max(g["e_max"] for g in learned)
    ref = torch.cat(db_dev)
    rbounds = [k * n for k in range(n_series + 1)]
    W = n - m + 1
    V = valid_windows(dbounds, m)
    t0 = time.perf_counter()
    joined = [abjoin.ab_join(q, D, dbounds, m) for q in held_dev]
    torch.cuda.synchronize()
    t_join = time.perf_counter() - t0
    t0 = time.perf_counter()
    found = [abjoin.discords(q, Ph, e_max, ref, rbounds, m, K) for q, (Ph, _) in zip(held_dev, joined)]
    torch.cuda.synchronize()
    t_disc = time.perf_counter() - t0
    hits = 0
    for (_, starts), r in zip(held, found):
        for row in r["rows"]:
            hits += int(np.any(np.abs(starts - int(row)) <= 260))
    # for the CPU leg's check: the first held-out series, its dictionary join
    # and its discords, with the dictionary and the database on the host
    check = (held[0][0], D.cpu().numpy(), np.asarray(dbounds), np.concatenate(db), np.asarray(rbounds), m,
             joined[0][0].cpu().numpy().astype(np.float64), joined[0][1].cpu().numpy(), found[0])
    return check, {"database": f"{n_series} x {n} ECG-like", "held_out": f"{n_series} x {n}, 50 planted beats each",
            "m": m, "space_saving": space_saving, "K": K,
            "dictionary_samples": int(D.numel()), "dictionary_segments": len(dbounds) - 1, "e_max": e_max,
            "learn_ms_per_series": t_learn * 1e3 / n_series,
            "join_ms_per_series": t_join * 1e3 / n_series, "join_pairs_per_s": n_series * W * V / t_join,
            "discords_ms_per_series": t_disc * 1e3 / n_series,
            "exact_rows_fraction": float(np.mean([r["rows_exact"] / W for r in found])),
            "rounds": [int(r["rounds"]) for r in found], "certified_bits": [int(r["certified"]) for r in found],
            "discords_on_planted_beats": f"{hits} of {n_series * K}"}


def pipeline_errors(record, check, threads, rows=256):
    """The first held-out series against the FP64 oracle: its dictionary join
    on `rows` random rows, and its discords' values (exact distances to the
    whole database) at the rows returned."""
    import oracle

    q, D, dbounds, ref, rbounds, m, Ph, Ih, found = check
    W = len(q) - m + 1
    sample = np.sort(np.random.default_rng(77).choice(W, rows, replace=False))
    Po, Io, P2o = oracle.ab_join(q, D, dbounds, m, rows=sample, threads=threads, second=True)
    clear = (P2o - Po) > 1e-3
    record["dictionary_join_vs_oracle"] = {
        "rows": rows, "max_abs": float(np.abs(Ph[sample] - Po).max()),
        "index_match_clear_rows": float(np.mean(Ih[sample][clear] == Io[clear])) if clear.any() else 1.0}
    drows = np.asarray(found["rows"], dtype=np.int64)
    Pd, _ = oracle.ab_join(q, ref, rbounds, m, rows=np.sort(drows), threads=threads)
    order = np.argsort(drows)
    got = np.asarray(found["values"], dtype=np.float64)[order]
    record["discord_values_vs_oracle"] = {"rows": int(len(drows)), "max_abs": float(np.abs(got - Pd).max())}


def time_tier(abjoin, q, d, bounds, m, tier, steps, warmup, P, I):
    import torch

    for _ in range(warmup):
        abjoin.ab_join(q, d, bounds, m, tier=tier, out=(P, I))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        abjoin.ab_join(q, d, bounds, m, tier=tier, out=(P, I))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def serving(abjoin, synth, tiers, n_req: int, fracs=(0.5, 0.8, 0.95)):
    """Serving workload: a resident dictionary of 64 x 1,000 ECG-like samples;
    requests with log-uniform lengths in [1,024, 65,536] and m drawn from
    {64, 128, 256}.  Saturation throughput first (all requests at once), then
    Poisson arrivals at fractions of the saturation rate; p50/p99 latency from
    submit to results on the host."""
    import threading

    w = synth.WORKLOADS["serve_dict64x1000"]()
    dct = abjoin.Dictionary(w["dict"], w["bounds"], (64, 128, 256))
    pool = synth.ecg_like(1 << 22, synth.rng_for(3, 0))
    out = {"workload": "serve_dict64x1000", "requests": n_req, "dict_segments": 64, "segment_samples": 1000,
           "query_samples": "log-uniform 1024..65536", "m": [64, 128, 256], "tiers": {}}
    for tier in tiers:
        def run(qps):
            sched = synth.serving_schedule(n_req, qps if qps else 1e9, synth.rng_for(4, int(qps or 0)))
            offs = synth.rng_for(4, 99).integers(0, len(pool) - 65536, n_req)
            srv = abjoin.Server(dct, tier=tier, max_slots=512, mem_budget=2 << 30)
            ids = [None] * n_req
            t0 = time.perf_counter()

            def feeder():
                for k, r in enumerate(sched):
                    if qps:
                        dt = r.arrival_s - (time.perf_counter() - t0)
                        if dt > 0:
                            time.sleep(dt)
                    ids[k] = srv.submit(pool[offs[k]:offs[k] + r.length], r.m)

            th = threading.Thread(target=feeder)
            th.start()
            th.join()
            assert srv.drain(600000) == abjoin.ABJ_OK
            st = srv.stats()
            for i in ids:
                srv.result(i)
            srv.close()
            return st

        sat = run(None)
        sat_qps = sat["completed"] / sat["busy_s"]
        rec = {"saturation_pairs_per_s": sat["pairs"] / sat["busy_s"], "saturation_qps": sat_qps,
               "batches": sat["batches"], "levels": []}
        for f in fracs:
            st = run(f * sat_qps)
            rec["levels"].append({"qps": f * sat_qps, "load": f, "p50_ms": st["p50_s"] * 1e3,
                                  "p99_ms": st["p99_s"] * 1e3, "max_ms": st["max_s"] * 1e3,
                                  "pairs_per_s": st["pairs"] / st["busy_s"], "batches": st["batches"]})
        out["tiers"][tier] = rec
    dct.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tier", default="fp32", choices=["fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tiers", action="store_true", help="skip the BF16/FP16 comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--no-pipeline", action="store_true", help="skip the learning + join + discords pipeline")
    ap.add_argument("--workload", default=WORKLOAD, choices=[WORKLOAD, "rw1m_m128"],
                    help="the timed join: the dictionary workload (default) or 1M x 1M random walks at m = 128")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the timed steps, run one device-to-device copy of this many bytes "
                         "(reference dispatch for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2112_12965_amd import abjoin, synth

    w = synth.WORKLOADS[args.workload]()
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
    achieved = FLOPS_PER_PAIR * kernel_pairs / (kernel_ms * 1e-3)
    src = os.path.join(ROOT, "paper_2112_12965_amd", "csrc", "join_fp32.hip")

    def prof(kind):
        return os.path.join(ROOT, "profiles", f"k_join_fp32_{args.workload}_{kind}_counters.md")

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
        "config": {"workload": args.workload, "query_samples": len(w["query"]), "dict_segments": len(bounds) - 1,
                   "segment_samples": int(bounds[1] - bounds[0]), "m": m, "tier": args.tier,
                   "pairs_per_step": pairs},
        "roofline": {"bound": "alu", "kernel": "k_join_fp32", "achieved": achieved / 1e12,
                     "peak": FP32_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK, "flops_per_pair": FLOPS_PER_PAIR,
                     "kernel_ms": kernel_ms,
                     "traffic": profiled_field(src, prof("hbm"), "traffic_bytes_per_launch")},
    }
    # the same kernel against the issue ceiling of its FMA-class instructions,
    # with their lane-instructions per pair (FP64 edges included) from the
    # committed counters; the other VALU instructions (maxima, selects, the DPP
    # add) are listed too, but some of them issue faster than 16 lanes a clock
    fpp = profiled_field(src, prof("valu_types"), "fma_class_lane_instructions_per_pair")
    vpp = profiled_field(src, prof("valu_types"), "valu_lane_instructions_per_pair")
    out["roofline"]["valu_issue"] = None if fpp is None else {
        "fma_class_lane_instructions_per_pair": fpp, "all_valu_lane_instructions_per_pair": vpp,
        "ceiling_lane_instructions_per_s": VALU_LANE_INSTR_PER_S,
        "frac": kernel_pairs / (kernel_ms * 1e-3) * fpp / VALU_LANE_INSTR_PER_S}
    results = {"fp32": (P.cpu().numpy(), I.cpu().numpy())}
    if not args.no_tiers:
        out["tiers"] = {"fp32": {"pairs_per_s": out["value"], "ms_per_step": out["ms_per_step"]}}
        for tier in ("bf16", "fp16"):
            Pt = torch.empty_like(P)
            It = torch.empty_like(I)
            dtt = time_tier(abjoin, q, d, bounds, m, tier, max(args.steps // 5, 3), 2, Pt, It)
            out["tiers"][tier] = {"pairs_per_s": pairs / dtt, "ms_per_step": dtt * 1e3,
                                  "vs_fp32": (pairs / dtt) / out["value"]}
            results[tier] = (Pt.cpu().numpy(), It.cpu().numpy())
        # the precision tier against the FP32 tier where its O(m) products are short
        out["tiers_short_windows"], short_data = short_windows(abjoin, synth)
    if not args.no_pipeline:
        pipe_check, out["pipeline"] = pipeline(abjoin, synth)
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        cb, errs = cpu_baseline(w, results, args.cpu_seconds, threads)
        out["cpu_baseline"] = cb
        out["error_vs_oracle"] = errs
        if not args.no_tiers:
            short_window_errors(out["tiers_short_windows"], short_data, threads)
        if not args.no_pipeline:
            pipeline_errors(out["pipeline"], pipe_check, threads)
    if not args.no_serving:
        out["serving"] = serving(abjoin, synth, ("fp32", "bf16"), args.serve_requests)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
