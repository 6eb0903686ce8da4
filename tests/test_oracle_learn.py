"""Pins for the oracle of the learning phase (Alg. 1)."""
import math

import numpy as np
import pytest

from oracle import learn
from paper_2112_12965_amd import synth


def two_pattern_series(seed=0, n=6000, m=64):
    """Random-walk background with pattern V (5 copies) and pattern C (3 copies)."""
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.standard_normal(n)) * 0.3
    t = np.linspace(-1, 1, m)
    V = 8 * np.abs(t)
    C = 8 * np.where(np.abs(t) < 0.5, np.cos(6 * np.pi * t), -np.abs(t))
    starts_v = [500, 1700, 2900, 4100, 5300]
    starts_c = [1100, 2300, 3500]
    for s in starts_v:
        x[s:s + m] = V + rng.normal(0, 0.02, m) + x[s]
    for s in starts_c:
        x[s:s + m] = C + rng.normal(0, 0.02, m) + x[s]
    return x, starts_v, starts_c


def test_first_elements_are_distinct_motifs():
    """Fig. 4: after the first motif is added, subtracting its distance profile
    demotes its repeats, so the next element is the other motif."""
    m = 64
    x, sv, sc = two_pattern_series(m=m)
    r = learn.learn_dictionary(x, m, k=1.5, stop="space_saving", value=0.9)
    near = lambda j, starts: min(abs(j - s) for s in starts) <= 3
    j1, j2 = r["chosen"][:2]
    kinds = ["V" if near(j, sv) else "C" if near(j, sc) else "?" for j in (j1, j2)]
    assert set(kinds) == {"V", "C"}, (r["chosen"][:4], kinds)


@pytest.mark.parametrize("value", [0.95, 0.8, 0.5])
def test_space_saving_stop_and_structure(value):
    m, k = 32, 1.5
    x = synth.ecg_like(4000, np.random.default_rng(3))
    r = learn.learn_dictionary(x, m, k=k, stop="space_saving", value=value)
    n = len(x)
    segs = r["segments"]
    size = sum(b - a for a, b in segs)
    assert size >= (1 - value) * n  # stopped only once the budget was reached
    # one element earlier the budget was not reached
    prev = learn.merge_elements([learn.element_of(j, n, m, k) for j in r["chosen"][:-1]])
    assert sum(b - a for a, b in prev) < (1 - value) * n
    # Prop. 1: every dictionary element is a verbatim slice of T_B
    for (a, b), lo, hi in zip(segs, r["bounds"][:-1], r["bounds"][1:]):
        np.testing.assert_array_equal(r["dictionary"][lo:hi], x[a:b])
    assert all(b1 < a2 for (_, b1), (a2, _) in zip(segs, segs[1:]))  # merged: disjoint, not touching
    # exclusion zone: chosen windows are more than floor(m/2) apart
    ch = np.array(r["chosen"])
    d = np.abs(ch[:, None] - ch[None, :]) + np.eye(len(ch), dtype=int) * 10 ** 9
    assert d.min() > m // 2
    # context: every chosen window lies inside one segment
    for j in ch:
        assert any(a <= j and j + m <= b for a, b in segs)


def test_e_max_stop_and_monotonicity():
    m = 32
    x = synth.ecg_like(3000, np.random.default_rng(4))
    target = 3.0
    r = learn.learn_dictionary(x, m, stop="e_max", value=target)
    assert r["e_max"] <= target
    prev = learn.merge_elements([learn.element_of(j, len(x), m, 1.5) for j in r["chosen"][:-1]])
    assert learn.e_max_of(x, prev, m) > target  # it stopped at the first dictionary meeting the bound
    # larger dictionaries (prefixes of the same greedy sequence) never have larger e_max
    e = [learn.e_max_of(x, learn.merge_elements([learn.element_of(j, len(x), m, 1.5) for j in r["chosen"][:t]]), m)
         for t in range(1, len(r["chosen"]) + 1)]
    assert all(b <= a + 1e-12 for a, b in zip(e, e[1:]))


def test_lemmas_hold_for_a_learned_dictionary(orc):
    m = 48
    tb = synth.ecg_like(5000, np.random.default_rng(5))
    ta = synth.ecg_like(3000, np.random.default_rng(6), n_anomalies=3)
    r = learn.learn_dictionary(tb, m, stop="space_saving", value=0.8)
    Phat, _ = orc.ab_join(ta, r["dictionary"], r["bounds"], m)
    P, _ = orc.ab_join(ta, tb, [0, len(tb)], m)
    assert np.all(Phat >= P - 1e-12)                 # Lemma 1
    assert np.all(Phat - P <= r["e_max"] + 1e-12)    # Lemma 2


def test_forced_replay_checks_choices():
    m = 32
    x = synth.ecg_like(2500, np.random.default_rng(7))
    r = learn.learn_dictionary(x, m, stop="space_saving", value=0.9)
    r2 = learn.learn_dictionary(x, m, stop="space_saving", value=0.9, forced=r["chosen"])
    assert r2["chosen"] == r["chosen"] and r2["segments"] == r["segments"]
    bad = list(r["chosen"])
    bad[1] = (bad[1] + 500) % (len(x) - m)
    with pytest.raises(AssertionError):
        learn.learn_dictionary(x, m, stop="space_saving", value=0.9, forced=bad)
    with pytest.raises(AssertionError):
        learn.learn_dictionary(x, m, stop="space_saving", value=0.9, forced=r["chosen"][:-1])


def test_element_of_matches_hand_derived_golden():
    """Alg. 1's context window (Sec. 3.1) against values worked out by hand
    (tests/golden/element_of.json): total length ceil(k m) bounded by [m, n],
    the chosen window centred with the odd sample after it, shifted inside the
    series at both ends."""
    import json
    import os

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "element_of.json")))
    assert len(g["cases"]) >= 10
    for c in g["cases"]:
        got = learn.element_of(c["j"], c["n"], c["m"], c["k"])
        assert list(got) == c["expect"], (c, got)
        a, b = got
        # structural facts that hold for every case: the window is inside its element
        assert a <= c["j"] and c["j"] + c["m"] <= b and 0 <= a and b <= c["n"]


@pytest.mark.parametrize("seed", range(6))
def test_merge_elements_is_the_union_of_the_intervals(seed):
    """Alg. 1's merge: the segments cover exactly the union of the elements,
    sorted, and no two of them overlap or touch (reading 10)."""
    rng = np.random.default_rng(seed)
    n = 300
    els = []
    for _ in range(int(rng.integers(1, 12))):
        a = int(rng.integers(0, n - 5))
        els.append((a, int(min(n, a + rng.integers(1, 40)))))
    segs = learn.merge_elements(els)
    cover = np.zeros(n + 1, dtype=bool)
    for a, b in els:
        cover[a:b] = True
    got = np.zeros(n + 1, dtype=bool)
    for a, b in segs:
        assert a < b and not got[a:b].any()
        got[a:b] = True
    assert np.array_equal(got, cover)
    assert all(b1 < a2 for (_, b1), (a2, _) in zip(segs, segs[1:]))  # gaps between segments, in order


def test_e_max_of_matches_brute_force():
    """Def. 10 by plain loops: the largest, over the windows of T, of the
    distance to the nearest window that lies inside one dictionary segment."""
    rng = np.random.default_rng(8)
    m = 6
    T = np.cumsum(rng.standard_normal(90))
    segs = [(3, 20), (40, 47), (60, 88)]

    def z(w):
        return (w - w.mean()) / w.std()

    dwin = [T[j:j + m] for a, b in segs for j in range(a, b - m + 1)]
    best = [min(np.sqrt(np.sum((z(T[i:i + m]) - z(v)) ** 2)) for v in dwin) for i in range(len(T) - m + 1)]
    assert abs(learn.e_max_of(T, segs, m) - max(best)) < 1e-9
