"""Pins for the FP64 oracle: each test ties it to something other than itself.

Routes used (all CPU, no GPU):
  * hand-derived closed forms for tiny windows (tests/golden/zdist_m3.json);
  * scipy: cdist over scipy.stats.zscore(ddof=0) windows (an independent
    implementation of Def. 4 + Def. 7), and numpy corrcoef -> sqrt(2m(1-rho));
  * a pure-Python brute force written from the definitions with numpy mean/std;
  * invariants the paper proves or states: Alg. 2's decomposition into per-element
    joins, Prop. 1 / Lemma 1 (no false negatives), Lemma 2 (error <= e_max),
    affine invariance of z-normalisation, range [0, 2 sqrt(m)].
"""
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st
from numpy.lib.stride_tricks import sliding_window_view
from scipy.spatial.distance import cdist
from scipy.stats import zscore

from paper_2112_12965_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _valid_mask(bounds, n, m):
    v = np.zeros(n - m + 1, bool)
    for s in range(len(bounds) - 1):
        lo, hi = int(bounds[s]), int(bounds[s + 1]) - m + 1
        if hi > lo:
            v[lo:hi] = True
    return v


def scipy_join(a, b, bounds, m):
    """Independent route: scipy z-score (population) windows + cdist, masked columns."""
    ZA = zscore(sliding_window_view(a, m), axis=1, ddof=0)
    ZB = zscore(sliding_window_view(b, m), axis=1, ddof=0)
    D = cdist(ZA, ZB)
    D[:, ~_valid_mask(bounds, len(b), m)] = np.inf
    return D.min(1), D.argmin(1), D


def python_brute(a, b, bounds, m):
    """Pure-Python loops over the definitions (tiny inputs only)."""
    valid = _valid_mask(bounds, len(b), m)
    P, I = [], []
    for i in range(len(a) - m + 1):
        u = np.asarray(a[i:i + m], float)
        zu = (u - u.mean()) / u.std()
        best, arg = math.inf, -1
        for j in range(len(b) - m + 1):
            if not valid[j]:
                continue
            v = np.asarray(b[j:j + m], float)
            zv = (v - v.mean()) / v.std()
            dist = math.sqrt(sum((x - y) ** 2 for x, y in zip(zu, zv)))
            if dist < best:
                best, arg = dist, j
        P.append(best)
        I.append(arg)
    return np.array(P), np.array(I)


# ---------------------------------------------------------------- golden values
def test_golden_hand_derived(orc):
    g = json.load(open(os.path.join(GOLDEN, "zdist_m3.json")))
    m = g["m"]
    for case in g["cases"]:
        P, I, P2 = orc.ab_join(case["query"], case["dict"], case["bounds"], m, second=True)
        for row in case["rows"]:
            i = row["i"]
            want = math.inf if row["P"] == "inf" else float(row["P"])
            if "dot" in row:  # closed form from the integer deviation vectors
                cf = math.sqrt(2 * m * (1 - row["dot"] / math.sqrt(row["nu"] * row["nv"])))
                assert cf == pytest.approx(want, abs=1e-15)
            if math.isinf(want):
                assert math.isinf(P[i]), case["name"]
            else:
                assert P[i] == pytest.approx(want, abs=1e-12), case["name"]
            assert I[i] == row["I"], case["name"]
            if "second" in row:
                assert P2[i] == pytest.approx(row["second"]["P2"], abs=1e-12), case["name"]


# ---------------------------------------------------------------- library routes
@pytest.mark.parametrize("m", [3, 8, 16])
def test_matches_scipy_zscore_cdist(orc, m):
    rng = np.random.default_rng(100 + m)
    a = rng.standard_normal(257).cumsum()
    b = rng.standard_normal(301).cumsum()
    bounds = [0, 90, 91, 200, 301]  # includes a segment shorter than m
    P, I = orc.ab_join(a, b, bounds, m)
    Ps, Is, _ = scipy_join(a, b, bounds, m)
    np.testing.assert_allclose(P, Ps, rtol=0, atol=1e-10)
    np.testing.assert_array_equal(I, Is)


def test_matches_python_brute(orc):
    rng = np.random.default_rng(7)
    a = rng.standard_normal(40)
    b = rng.standard_normal(50)
    bounds = [0, 17, 50]
    for m in (3, 5):
        P, I = orc.ab_join(a, b, bounds, m)
        Pp, Ip = python_brute(a, b, bounds, m)
        np.testing.assert_allclose(P, Pp, rtol=0, atol=1e-12)
        np.testing.assert_array_equal(I, Ip)


def test_closed_form_corrcoef(orc):
    """d = sqrt(2 m (1 - rho)) with rho from numpy's Pearson correlation."""
    rng = np.random.default_rng(11)
    m = 64
    a = rng.standard_normal(600).cumsum()
    b = rng.standard_normal(500).cumsum()
    ii = rng.integers(0, len(a) - m + 1, 200)
    jj = rng.integers(0, len(b) - m + 1, 200)
    d = orc.pair_dists(a, b, m, ii, jj)
    rho = np.array([np.corrcoef(a[i:i + m], b[j:j + m])[0, 1] for i, j in zip(ii, jj)])
    np.testing.assert_allclose(d, np.sqrt(2 * m * (1 - rho)), rtol=0, atol=1e-9)


def test_window_stats_against_numpy(orc):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(1000).cumsum() + 1e3
    m = 37
    mu, sd, flat, bad = orc.window_stats(x, m)
    W = sliding_window_view(x, m)
    np.testing.assert_allclose(mu, W.mean(1), rtol=1e-14)
    np.testing.assert_allclose(sd, W.std(1, ddof=0), rtol=1e-12)
    assert not flat.any() and not bad.any()


@settings(max_examples=60, deadline=None, derandomize=True)
@given(
    seed=st.integers(0, 2**31 - 1),
    m=st.integers(2, 12),
    na=st.integers(12, 60),
    cuts=st.lists(st.integers(1, 25), min_size=1, max_size=5),
)
def test_property_random_layouts(orc, seed, m, na, cuts):
    """Exhaustive pairs on tiny random inputs and random segment layouts."""
    rng = np.random.default_rng(seed)
    bounds = np.concatenate([[0], np.cumsum(cuts)])
    nb = int(bounds[-1])
    if na < m or nb < m:
        return
    a = rng.standard_normal(na)
    b = rng.standard_normal(nb)
    P, I = orc.ab_join(a, b, bounds, m)
    Ps, Is, D = scipy_join(a, b, bounds, m)
    np.testing.assert_allclose(P, Ps, rtol=0, atol=1e-10)
    # index: exact wherever the best is unique by a margin
    srt = np.sort(D, axis=1)
    with np.errstate(invalid="ignore"):
        clear = (srt[:, 1] - srt[:, 0] > 1e-9) if D.shape[1] > 1 else np.ones(len(P), bool)
    clear &= np.isfinite(Ps)
    np.testing.assert_array_equal(I[clear], Is[clear])
    assert np.all(I[np.isinf(Ps)] == -1)
    assert np.all((P[np.isfinite(P)] >= 0) & (P[np.isfinite(P)] <= 2 * math.sqrt(m) + 1e-12))


# ---------------------------------------------------------------- invariants
def test_segment_boundary_exact(orc):
    """A window ending exactly at a break is valid; one sample further is not (Def. 8)."""
    m = 4
    rng = np.random.default_rng(5)
    b = rng.standard_normal(20)
    bounds = [0, 10, 20]
    valid = orc.valid_windows(bounds, 20, m)
    assert valid[6] and not valid[7] and not valid[9] and valid[10] and valid[16]
    # plant window 6 (last valid of segment 0) and window 7 (first masked) into the query
    a = np.concatenate([b[6:10], rng.standard_normal(3), 2.0 * b[7:11] + 1.0])
    P, I = orc.ab_join(a, b, bounds, m)
    assert P[0] < 1e-7 and I[0] == 6
    assert I[7] != 7 and P[7] > 1e-3


def test_decomposition_alg2(orc):
    """Alg. 2: joining the concatenation with masking = element-wise min of per-element joins."""
    rng = np.random.default_rng(21)
    m = 24
    a = synth.ecg_like(1500, rng)
    segs = [synth.ecg_like(L, rng) for L in (300, 500, 23, 410)]
    bounds = np.concatenate([[0], np.cumsum([len(s) for s in segs])])
    d = np.concatenate(segs)
    P, I = orc.ab_join(a, d, bounds, m)
    Pm = np.full(len(a) - m + 1, np.inf)
    Im = np.full(len(a) - m + 1, -1)
    for s, seg in enumerate(segs):
        if len(seg) < m:
            continue
        Ps, Is = orc.ab_join(a, seg, [0, len(seg)], m)
        better = Ps < Pm
        Pm[better] = Ps[better]
        Im[better] = Is[better] + bounds[s]
    np.testing.assert_array_equal(P, Pm)
    np.testing.assert_array_equal(I, Im)


def test_overlap_split_equivalence(orc):
    """Cutting T_B into pieces that overlap by m-1 keeps every window exactly once (Def. 8)."""
    rng = np.random.default_rng(8)
    m = 32
    tb = rng.standard_normal(1200).cumsum()
    ta = rng.standard_normal(700).cumsum()
    cuts = [0, 250, 251, 600, 1200 - m + 1]
    pieces, starts = [], []
    for s in range(len(cuts) - 1):
        pieces.append(tb[cuts[s]:cuts[s + 1] + m - 1])
        starts.append(cuts[s])
    bounds = np.concatenate([[0], np.cumsum([len(p) for p in pieces])])
    P1, I1 = orc.ab_join(ta, tb, [0, len(tb)], m)
    P2, I2 = orc.ab_join(ta, np.concatenate(pieces), bounds, m)
    np.testing.assert_array_equal(P1, P2)
    seg = np.searchsorted(bounds, I2, side="right") - 1
    np.testing.assert_array_equal(I1, I2 - bounds[seg] + np.asarray(starts)[seg])


def test_lemma1_and_lemma2(orc):
    """Prop. 1 + Lemma 1: P_hat >= P;  Lemma 2: P_hat - P <= e_max (Def. 10)."""
    rng = np.random.default_rng(42)
    m = 32
    tb = rng.standard_normal(3000).cumsum()
    ta = rng.standard_normal(1500).cumsum()
    offs = [100, 1200, 2500]
    dct = np.concatenate([tb[o:o + 300] for o in offs])
    bounds = [0, 300, 600, 900]
    Phat, _ = orc.ab_join(ta, dct, bounds, m)
    P, _ = orc.ab_join(ta, tb, [0, len(tb)], m)
    e_max = orc.ab_join(tb, dct, bounds, m)[0].max()
    assert np.all(Phat >= P - 1e-12)
    assert np.all(Phat - P <= e_max + 1e-12)
    assert (Phat - P).max() > 0  # the dictionary is a real approximation here


def test_transpose_consistency(orc):
    rng = np.random.default_rng(9)
    m = 10
    a = rng.standard_normal(90).cumsum()
    b = rng.standard_normal(130).cumsum()
    D = orc.dist_matrix(a, b, m)
    Pab, Iab = orc.ab_join(a, b, [0, len(b)], m)
    Pba, Iba = orc.ab_join(b, a, [0, len(a)], m)
    np.testing.assert_array_equal(Pab, D.min(1))
    np.testing.assert_array_equal(Pba, D.min(0))
    np.testing.assert_array_equal(Iab, D.argmin(1))
    np.testing.assert_array_equal(Iba, D.argmin(0))


def test_planted_affine_copies(orc):
    """z-normalisation is affine invariant: alpha*x+beta (alpha>0) is at distance 0,
    alpha<0 at exactly 2 sqrt(m) (rho = -1)."""
    rng = np.random.default_rng(13)
    m = 100
    b = synth.random_walk(2000, rng)
    a = synth.random_walk(2000, rng)
    j = 777
    a[300:300 + m] = 3.5 * b[j:j + m] - 40.0
    a[1500:1500 + m] = -0.25 * b[j:j + m] + 7.0
    P, I = orc.ab_join(a, b, [0, len(b)], m)
    assert P[300] < 1e-9 and I[300] == j
    d_neg = orc.pair_dists(a, b, m, [1500], [j])[0]
    assert d_neg == pytest.approx(2 * math.sqrt(m), abs=1e-9)
    assert np.all((P >= 0) & (P <= 2 * math.sqrt(m) + 1e-12))


def test_ties_pick_smallest_index(orc):
    rng = np.random.default_rng(17)
    m = 16
    seg = rng.standard_normal(100)
    d = np.concatenate([seg, seg])  # every window appears twice, bitwise equal
    a = rng.standard_normal(80)
    P, I = orc.ab_join(a, d, [0, 100, 200], m)
    assert np.all(I < 100 - m + 1)


def test_flat_and_nonfinite_conventions(orc):
    m = 8
    rng = np.random.default_rng(19)
    q = rng.standard_normal(60)
    q[10:30] = 2.5  # flat query windows 10..22
    q[45] = np.nan  # rows 38..45 have a non-finite sample
    d = rng.standard_normal(80)
    d[50:60] = -1.0  # flat reference windows 50..52
    d[5] = np.inf  # reference windows 0..5 are not windows
    P, I = orc.ab_join(q, d, [0, 80], m)
    assert np.all(P[10:23] == 0) and np.all(I[10:23] == 50)
    assert np.all(np.isnan(P[38:46])) and np.all(I[38:46] == -1)
    assert np.all(I[np.isfinite(P)] > 5)
    nonflat = [i for i in range(len(P)) if np.isfinite(P[i]) and not (10 <= i <= 22)]
    assert np.all(P[nonflat] <= math.sqrt(m) + 1e-12)  # a flat window is always at sqrt(m)
    # without the flat reference stretch, a flat row is at sqrt(m) from everything: first valid index
    d2 = d.copy()
    d2[50:60] = rng.standard_normal(10)
    P2, I2 = orc.ab_join(q, d2, [0, 80], m)
    assert np.all(P2[10:23] == pytest.approx(math.sqrt(m))) and np.all(I2[10:23] == 6)


def test_invalid_arguments(orc):
    with pytest.raises(ValueError):
        orc.ab_join(np.zeros(10), np.zeros(10), [0, 5, 5, 10], 3)  # non-increasing bounds
    with pytest.raises(ValueError):
        orc.ab_join(np.zeros(10), np.zeros(10), [0, 9], 3)  # does not end at n
    with pytest.raises(ValueError):
        orc.ab_join(np.zeros(2), np.zeros(10), [0, 10], 3)  # query shorter than m


# ---------------------------------------------------------------- learning-phase primitives
def test_self_join_matches_scipy_with_exclusion(orc):
    """Alg. 1's P_B: intra-join with trivial-match exclusion |i - j| <= floor(m/2)."""
    rng = np.random.default_rng(31)
    for m in (4, 9, 32):
        x = rng.standard_normal(400).cumsum()
        P, I = orc.self_join(x, m)
        Z = zscore(sliding_window_view(x, m), axis=1, ddof=0)
        D = cdist(Z, Z)
        W = len(D)
        ii, jj = np.indices((W, W))
        D[np.abs(ii - jj) <= m // 2] = np.inf
        np.testing.assert_allclose(P, D.min(1), rtol=0, atol=1e-10)
        np.testing.assert_array_equal(I, D.argmin(1))
        assert np.all(np.abs(I - np.arange(W)) > m // 2)


def test_self_join_exclusion_boundary(orc):
    """A copy exactly floor(m/2)+1 away is found; one exactly floor(m/2) away is excluded."""
    rng = np.random.default_rng(32)
    m = 10
    x = rng.standard_normal(200)
    x[100:110] = x[50:60]  # window 100 copies window 50
    P, I = orc.self_join(x, m)
    assert P[50] < 1e-9 and I[50] == 100
    y = rng.standard_normal(200)
    y[55:65] = 3.0 * y[50:60] + 1.0  # 5 = floor(m/2) apart: a trivial match
    P, I = orc.self_join(y, m)
    assert I[50] != 55 and P[50] > 1e-3


def test_dist_profile_matches_scipy(orc):
    """Def. 4 distance profile of one query window against every window of x."""
    rng = np.random.default_rng(33)
    m = 24
    x = rng.standard_normal(500).cumsum()
    w = x[123:123 + m].copy()
    S = orc.dist_profile(x, m, w)
    Z = zscore(sliding_window_view(x, m), axis=1, ddof=0)
    zw = zscore(w, ddof=0)
    np.testing.assert_allclose(S, np.sqrt(((Z - zw) ** 2).sum(1)), rtol=0, atol=1e-10)
    assert S[123] < 1e-12
