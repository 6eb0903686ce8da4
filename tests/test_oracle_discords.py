"""Pins for the discord oracle.

* the greedy top-K equals an independent sort-and-scan selection on random
  profiles with ties, NaN and inf;
* K = 1 is the argmax of the finite entries;
* planted bursts in a periodic series are what the exact discords find;
* certification: whenever the test passes, the exact discord is where the
  approximate profile says (Lemmas 1 and 2 make this a theorem; the data
  make it a check of the oracle's join, greedy and e_max together).
"""
import numpy as np
import pytest

from oracle import discords, learn


def sort_scan(P, K, excl):
    """Scan rows by decreasing value (ties: smaller index first), keeping each
    row farther than excl from every row kept so far."""
    P = np.asarray(P, dtype=np.float64)
    order = sorted(np.flatnonzero(np.isfinite(P)), key=lambda r: (-P[r], r))
    kept = []
    for r in order:
        if len(kept) == K:
            break
        if all(abs(r - k) > excl for k in kept):
            kept.append(int(r))
    return kept


@pytest.mark.parametrize("seed", range(12))
def test_greedy_matches_sort_scan(seed):
    rng = np.random.default_rng(seed)
    W = int(rng.integers(1, 300))
    P = np.round(rng.uniform(0, 5, W), 1)  # many exact ties
    P[rng.random(W) < 0.05] = np.nan
    P[rng.random(W) < 0.03] = np.inf
    K, excl = int(rng.integers(1, 12)), int(rng.integers(0, 20))
    rows, vals = discords.topk_discords(P, K, excl)
    assert list(rows) == sort_scan(P, K, excl)
    assert np.array_equal(vals, P[rows])


def test_k1_is_finite_argmax():
    P = np.array([1.0, np.inf, 3.0, np.nan, 3.0, 2.0])
    rows, vals = discords.topk_discords(P, 1, 0)
    assert list(rows) == [2] and vals[0] == 3.0
    assert discords.topk_discords(np.array([np.nan, np.inf]), 3, 0)[0].size == 0


def periodic(n, rng, bursts=(), amp=0.15):
    t = np.arange(n) + rng.uniform(0, 1000)
    x = np.sin(2 * np.pi * t / 100) + 0.4 * np.sin(2 * np.pi * t / 37) + rng.normal(0, 0.02, n)
    for b in bursts:
        x[b:b + 60] += np.cumsum(rng.normal(0, amp, 60))
    return x


@pytest.mark.parametrize("seed", range(3))
def test_planted_bursts_are_the_discords(orc, seed):
    rng = np.random.default_rng(seed)
    m = 128
    ref = periodic(6000, rng)
    bursts = [3000, 9000, 15000]
    q = periodic(20000, rng, bursts)
    rows, vals, nn = discords.exact_discords(q, ref, [0, len(ref)], m, 3)
    for r in rows:
        assert min(abs(r - b) for b in bursts) < m, (rows, vals)
    assert np.all(np.diff(vals) <= 0) and np.all(np.abs(np.diff(np.sort(rows))) > m - 1)


@pytest.mark.parametrize("seed", range(4))
def test_certification_guarantee(orc, seed):
    rng = np.random.default_rng(seed)
    m = 100
    ref = periodic(4000, rng)
    q = periodic(8000, rng, [5000], amp=0.5)
    r = learn.learn_dictionary(ref, m, stop="space_saving", value=0.3)
    Ph, _ = orc.ab_join(q, r["dictionary"], r["bounds"], m)
    P, _ = orc.ab_join(q, ref, [0, len(ref)], m)
    em = r["e_max"]
    assert np.all(P <= Ph + 1e-9) and np.all(Ph - em <= P + 1e-9)
    excl = m - 1
    top_hat = discords.topk_discords(Ph, 1, excl)[0][0]
    top = discords.topk_discords(P, 1, excl)[0][0]
    if discords.top_certified(Ph, em):
        assert top == top_hat
    if discords.top_certified(Ph, em, excl):
        assert abs(top - top_hat) <= excl
    # the literal test is the stricter one
    assert not discords.top_certified(Ph, em) or discords.top_certified(Ph, em, excl)


def test_certification_on_constructed_profiles():
    P = np.array([0.0, 5.0, 1.0, 0.5])
    assert discords.top_certified(P, 3.9) and not discords.top_certified(P, 4.0)
    P = np.array([5.0, 4.9, 0.0, 0.0, 1.0])
    assert not discords.top_certified(P, 1.0)
    assert discords.top_certified(P, 3.9, excl=1) and not discords.top_certified(P, 4.0, excl=1)
    assert discords.top_certified(np.array([2.0]), 10.0)
    assert not discords.top_certified(np.array([np.nan]), 0.0)
