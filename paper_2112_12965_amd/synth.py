"""Seeded synthetic inputs for the AB-join (matrix-profile inter-similarity join).

This module draws input series only.  It holds none of the join's arithmetic, so
both the FP64 CPU oracle (in the tests) and the HIP path take their inputs from
here without sharing any computation.

Every generator takes a ``numpy.random.Generator``; ``rng_for(cfg, role)`` builds
one from ``SeedSequence([cfg, role])`` so every workload is reproducible.
Roles: 0 = query / series A, 1 = reference / dictionary source B,
2 = anomaly placement, 3 = row sample, 4 = request arrivals and lengths.

The paper evaluates on random walks and on MIT-BIH ECG recordings
(Sec. 4.1, Sec. 4.3); the ECG data is not available here, so ``ecg_like`` is a
quasi-periodic stand-in built from Gaussian bumps.  Its shape parameters are a
choice made for this library, not values from the paper.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng_for",
    "random_walk",
    "ecg_like",
    "cut_dictionary",
    "ServingRequest",
    "serving_schedule",
    "WORKLOADS",
]


def rng_for(cfg: int, role: int) -> np.random.Generator:
    """Generator for workload ``cfg`` and input ``role`` (see module docstring)."""
    return np.random.default_rng(np.random.SeedSequence([int(cfg), int(role)]))


def random_walk(n: int, rng: np.random.Generator) -> np.ndarray:
    """Gaussian random walk: cumulative sum of N(0, 1) steps, float64, length n."""
    return np.cumsum(rng.standard_normal(int(n)))


# One normal beat as Gaussian bumps: (offset from the R peak as a fraction of the
# beat period, amplitude, width as a fraction of the period).  P, Q, R, S, T waves.
_NORMAL_BUMPS = (
    (-0.20, 0.15, 0.025),
    (-0.04, -0.12, 0.010),
    (0.00, 1.00, 0.012),
    (0.04, -0.25, 0.012),
    (0.30, 0.35, 0.050),
)


def _anomalous_bumps(kind: int):
    if kind == 0:  # ventricular-ectopic-like: no P wave, wide QRS, tall R, inverted T
        return (
            (-0.04, -0.12, 0.030),
            (0.00, 1.40, 0.036),
            (0.04, -0.25, 0.036),
            (0.30, -0.35, 0.050),
        )
    if kind == 1:  # tall, late T wave
        return (
            (-0.20, 0.15, 0.025),
            (-0.04, -0.12, 0.010),
            (0.00, 1.00, 0.012),
            (0.04, -0.25, 0.012),
            (0.35, 0.70, 0.050),
        )
    return _NORMAL_BUMPS  # kind 2: premature beat (normal shape, short period)


def ecg_like(
    n: int,
    rng: np.random.Generator,
    n_anomalies: int = 0,
    noise: float = 0.05,
    return_anomalies: bool = False,
):
    """Quasi-periodic ECG-like series of length n (float64).

    Beats follow each other with periods drawn from U[180, 260] samples; each beat
    is the sum of the five bumps in ``_NORMAL_BUMPS`` with the R peak at 0.4 of
    the beat; i.i.d. N(0, noise^2) noise is added.  ``n_anomalies`` beats (chosen
    uniformly, away from both ends) are replaced by one of three anomalous kinds:
    ectopic-like, tall late T, or premature (period x 0.6).  With
    ``return_anomalies`` the start sample of each anomalous beat is also returned
    (sorted int64 array).
    """
    n = int(n)
    # Draw enough beat periods to cover n samples even if every beat is short.
    nb = int(math.ceil(n / 180.0)) + 4
    periods = rng.uniform(180.0, 260.0, size=nb)
    kinds = np.full(nb, -1, dtype=np.int64)
    if n_anomalies:
        # Candidate beats must lie fully inside the series.
        n_full = int(np.searchsorted(np.cumsum(periods), n - 260.0))
        cand = np.arange(2, max(n_full - 2, 3))
        if len(cand) < n_anomalies:
            raise ValueError("series too short for the requested anomalies")
        pick = np.sort(rng.choice(cand, size=int(n_anomalies), replace=False))
        kinds[pick] = rng.integers(0, 3, size=int(n_anomalies))
        periods[kinds == 2] *= 0.6
    x = np.zeros(n, dtype=np.float64)
    starts = []
    s = 0.0
    for b in range(nb):
        p = periods[b]
        if s >= n:
            break
        c = s + 0.4 * p
        bumps = _NORMAL_BUMPS if kinds[b] < 0 else _anomalous_bumps(int(kinds[b]))
        lo = max(int(s - 0.2 * p), 0)
        hi = min(int(s + 1.4 * p) + 1, n)
        if hi > lo:
            t = np.arange(lo, hi, dtype=np.float64)
            for off, amp, wid in bumps:
                w = wid * p
                x[lo:hi] += amp * np.exp(-0.5 * ((t - (c + off * p)) / w) ** 2)
        if kinds[b] >= 0:
            starts.append(int(s))
        s += p
    x += rng.normal(0.0, noise, size=n)
    if return_anomalies:
        return x, np.asarray(starts, dtype=np.int64)
    return x


def cut_dictionary(src: np.ndarray, n_seg: int, seg_len: int, rng: np.random.Generator):
    """Cut ``n_seg`` non-overlapping pieces of ``seg_len`` samples from ``src``.

    ``src`` is split into ``n_seg`` equal blocks and one piece is taken at a
    uniformly random offset inside each block.  Returns ``(dict, seg_bounds,
    orig_start)``: the concatenation (float64), the CSR segment offsets
    ``[0, seg_len, ..., n_seg * seg_len]`` (int64) and each piece's start in
    ``src`` (int64).
    """
    block = len(src) // n_seg
    if block < seg_len:
        raise ValueError("source too short for the requested cuts")
    offs = rng.integers(0, block - seg_len + 1, size=n_seg)
    orig = np.arange(n_seg, dtype=np.int64) * block + offs
    pieces = [src[o : o + seg_len] for o in orig]
    bounds = np.arange(n_seg + 1, dtype=np.int64) * seg_len
    return np.concatenate(pieces).astype(np.float64), bounds, orig.astype(np.int64)


@dataclass(frozen=True)
class ServingRequest:
    arrival_s: float
    length: int
    m: int
    seed: int


def serving_schedule(n_req: int, qps: float, rng: np.random.Generator,
                     min_len: int = 1024, max_len: int = 65536, ms=(64, 128, 256)):
    """Request stream for the serving workload.

    Poisson arrivals at rate ``qps`` (exponential gaps), query lengths
    log-uniform on [min_len, max_len], window length uniform over ``ms``.
    """
    gaps = rng.exponential(1.0 / qps, size=n_req)
    arr = np.cumsum(gaps) - gaps[0]
    lens = np.rint(np.exp(rng.uniform(math.log(min_len), math.log(max_len), size=n_req))).astype(np.int64)
    mm = rng.choice(np.asarray(ms, dtype=np.int64), size=n_req)
    seeds = rng.integers(0, 2**31 - 1, size=n_req)
    return [ServingRequest(float(a), int(L), int(m), int(s)) for a, L, m, s in zip(arr, lens, mm, seeds)]


def _wl_small():
    """2,000-sample random walks A and B, m = 100 (plain exact join)."""
    a = random_walk(2000, rng_for(0, 0))
    b = random_walk(2000, rng_for(0, 1))
    return dict(query=a, dict=b, bounds=np.array([0, 2000], dtype=np.int64), m=100)


def _wl_dict_ecg():
    """ECG-like query of 131,072 samples (20 anomalous beats) against a dictionary
    of 16 x 2,000-sample cuts of a separate 262,144-sample draw, m = 256."""
    q, anom = ecg_like(131072, rng_for(1, 0), n_anomalies=20, return_anomalies=True)
    src = ecg_like(262144, rng_for(1, 1))
    d, bounds, orig = cut_dictionary(src, 16, 2000, rng_for(1, 2))
    return dict(query=q, dict=d, bounds=bounds, m=256, anomalies=anom, orig_start=orig)


def _wl_large_rw():
    """1,048,576-sample random walks A and B, m = 128 (precision-tier workload)."""
    a = random_walk(1 << 20, rng_for(2, 0))
    b = random_walk(1 << 20, rng_for(2, 1))
    return dict(query=a, dict=b, bounds=np.array([0, 1 << 20], dtype=np.int64), m=128)


def _wl_serving_dict():
    """Resident dictionary for serving: 64 x 1,000-sample ECG-like cuts."""
    src = ecg_like(64 * 4000, rng_for(3, 1))
    d, bounds, orig = cut_dictionary(src, 64, 1000, rng_for(3, 2))
    return dict(dict=d, bounds=bounds, orig_start=orig)


WORKLOADS = {
    "rw2k_m100": _wl_small,
    "ecg131k_dict16x2000_m256": _wl_dict_ecg,
    "rw1m_m128": _wl_large_rw,
    "serve_dict64x1000": _wl_serving_dict,
}
