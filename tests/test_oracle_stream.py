"""Pins for the streaming oracle (T2): the FP64 diagonal sweep of
``oracle/stream_oracle.c`` against the brute-force oracle, which the other pin
files tie to scipy, hand-derived values and the paper's invariants.

The two share no code: the sweep takes each row's column by an O(1)-per-pair
sliding dot product and then recomputes that column's distance directly, so on
every finite row its P equals the brute force's to rounding (1e-9 here) and
its I is the brute force's wherever the best-to-second gap is larger than
that; where the gap is smaller its I must still be a valid window whose
distance is within 1e-9 of the best.  Inputs cover segment layouts (Def. 8,
including segments shorter than m), flat stretches, non-finite samples,
planted copies (P = 0), and diagonals long enough for the periodic exact
restarts of the sweep.
"""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from paper_2112_12965_amd import synth

TOL = 1e-9


def check(q, d, bounds, m, rows=None):
    Ps, Is = oracle.ab_join_stream(q, d, bounds, m)
    Pb, Ib, P2b = oracle.ab_join(q, d, bounds, m, rows=rows, second=True)
    if rows is not None:
        Ps, Is = Ps[rows], Is[rows]
    r = np.arange(len(Pb)) if rows is None else np.asarray(rows)
    assert np.array_equal(np.isnan(Ps), np.isnan(Pb))
    assert np.array_equal(np.isinf(Ps), np.isinf(Pb))
    fin = np.isfinite(Pb)
    assert np.all(Is[~fin] == -1)
    err = np.abs(Ps[fin] - Pb[fin])
    assert err.size == 0 or err.max() <= TOL, err.max()
    with np.errstate(invalid="ignore"):
        clear = fin & (P2b - Pb > TOL)
    assert np.array_equal(Is[clear], Ib[clear]), np.flatnonzero(Is[clear] != Ib[clear])[:10]
    if fin.any():
        valid = oracle.valid_windows(bounds, len(d), m)
        assert valid[Is[fin]].all()
        dsel = oracle.pair_dists(q, d, m, r[fin], Is[fin])
        assert np.all(np.isfinite(dsel)) and np.max(dsel - Pb[fin]) <= TOL
    return dict(rows=int(len(Pb)), clear=int(clear.sum()))


@pytest.mark.parametrize("m", [2, 3, 16, 100])
def test_random_walk_one_segment(m):
    rng = np.random.default_rng(10 + m)
    q, d = synth.random_walk(1500, rng), synth.random_walk(1200, rng)
    st_ = check(q, d, [0, len(d)], m)
    if m >= 16:  # at m = 2 every z-normalised window is +-(1, -1): all rows tie
        assert st_["clear"] > 0.9 * st_["rows"]


@pytest.mark.parametrize("m", [8, 64, 200])
def test_segment_layouts(m):
    rng = np.random.default_rng(20 + m)
    q = synth.ecg_like(2500, rng, n_anomalies=1)
    d = synth.ecg_like(3000, rng)
    # a segment shorter than m (no window), one exactly m long (one window), a long one
    bounds = [0, 700, 700 + m - 1, 700 + m - 1 + m, 2100, 3000]
    check(q, d, bounds, m)


def test_many_short_segments():
    rng = np.random.default_rng(31)
    m = 32
    lens = rng.integers(20, 90, 60)
    d = synth.random_walk(int(lens.sum()), rng)
    bounds = np.concatenate([[0], np.cumsum(lens)])
    q = synth.random_walk(1000, rng)
    check(q, d, bounds, m)


def test_flat_nonfinite_and_planted_copies():
    rng = np.random.default_rng(41)
    m = 50
    q = synth.random_walk(1800, rng)
    d = synth.random_walk(1600, rng)
    q[200:200 + m] = 3.0 * d[900:900 + m] - 7.0       # planted copy: P = 0 at row 200
    q[600:700] = 4.0                                  # flat query stretch
    d[100:180] = -2.0                                 # flat dictionary stretch
    q[1000] = np.nan                                  # non-finite query sample
    d[1300] = np.inf                                  # non-finite dictionary sample
    P, I = oracle.ab_join_stream(q, d, [0, 800, 1600], m)
    assert P[200] < 1e-6 and I[200] == 900
    assert np.isnan(P[1000 - m + 1:1001]).all() and np.all(I[1000 - m + 1:1001] == -1)
    check(q, d, [0, 800, 1600], m)


def test_no_valid_window():
    rng = np.random.default_rng(43)
    q, d = rng.standard_normal(200), rng.standard_normal(90)
    P, I = oracle.ab_join_stream(q, d, [0, 30, 60, 90], 40)
    assert np.all(np.isinf(P)) and np.all(I == -1)
    check(q, d, [0, 30, 60, 90], 40)


def test_long_diagonals_with_large_offsets():
    """Diagonals of several thousand steps over a series far from zero: the
    restarts keep the sweep's choice exact on clear rows (brute force on a row
    sample)."""
    rng = np.random.default_rng(51)
    m = 128
    q = 1e4 + synth.random_walk(20000, rng)
    d = -3e3 + synth.random_walk(12000, rng)
    rows = np.sort(rng.choice(len(q) - m + 1, 300, replace=False))
    check(q, d, [0, len(d)], m, rows=rows)


@settings(max_examples=40, deadline=None)
@given(st.integers(0, 10 ** 6), st.integers(2, 12), st.integers(1, 4))
def test_hypothesis_tiny(seed, m, nseg):
    rng = np.random.default_rng(seed)
    nd = int(rng.integers(m, 120))
    nq = int(rng.integers(m, 100))
    d = np.round(rng.standard_normal(nd) * 3, 1)     # ties and flat windows happen
    q = np.round(rng.standard_normal(nq) * 3, 1)
    cuts = np.sort(rng.choice(np.arange(1, nd), size=min(nseg - 1, nd - 1), replace=False)) if nd > 1 else []
    bounds = np.concatenate([[0], cuts, [nd]]).astype(np.int64)
    check(q, d, bounds, m)
