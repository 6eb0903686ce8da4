"""GPU parity of the self-join and of the learning phase (Alg. 1).

Self-join: P within the FP32 bar (1e-3) of the FP64 oracle, NaN / inf rows
equal, every returned neighbour outside the trivial-match zone and within the
bar of the best; on small inputs the full distance matrix gives the
second-best distance, and I must equal the oracle's wherever the gap exceeds
the bar.

Learning phase: the oracle replays the GPU's choices (``forced``) and checks
at every step that the GPU's window is an argmin of the oracle's P' within
2e-3 (P_B carries the FP32 bar, S is FP64 on both sides), then must stop at the
same step; segments, offsets and dictionary samples must be identical and
e_max agree within the bar.
"""
import numpy as np
import pytest
import torch

from oracle import learn as olearn
from paper_2112_12965_amd import abjoin, synth

pytestmark = pytest.mark.gpu
TOL = 1e-3


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def gpu_self_join(x, m, excl=-1):
    P, I, P64 = abjoin.self_join(dev(x), m, excl)
    torch.cuda.synchronize()
    return P.cpu().numpy().astype(np.float64), I.cpu().numpy(), P64.cpu().numpy()


def check_self(orc, x, m, excl, exact_second=False):
    print(f"[case] self-join n={len(x)} m={m} excl={excl}", flush=True)
    P, I, P64 = gpu_self_join(x, m, excl)
    e = m // 2 if excl < 0 else excl
    Po, Io = orc.self_join(x, m, e)
    assert np.array_equal(np.isnan(P), np.isnan(Po)) and np.array_equal(np.isinf(P), np.isinf(Po))
    assert np.array_equal(np.isnan(P64), np.isnan(Po)) and np.array_equal(np.isinf(P64), np.isinf(Po))
    fin = np.isfinite(Po)
    assert np.all(I[~fin] == -1)
    err = np.abs(P[fin] - Po[fin])
    assert err.size == 0 or err.max() <= TOL, err.max()
    assert np.all(np.abs(P64[fin] - P[fin]) <= 1e-6 * np.maximum(1.0, P64[fin]))
    rows = np.flatnonzero(fin)
    assert np.all(np.abs(I[rows] - rows) > e), "returned a trivial match"
    if rows.size:
        dsel = orc.pair_dists(x, x, m, rows, I[rows])
        assert (dsel - Po[rows]).max() <= TOL
        assert np.allclose(dsel, P64[rows], atol=1e-9, rtol=0)
    if exact_second:
        D = orc.dist_matrix(x, x, m)
        W = D.shape[0]
        ii, jj = np.indices((W, W))
        D[np.abs(ii - jj) <= e] = np.inf
        D[np.isnan(D)] = np.inf
        srt = np.sort(D, axis=1)
        with np.errstate(invalid="ignore"):
            gap = srt[:, 1] - srt[:, 0]
            clear = fin & (gap > TOL)
        assert np.array_equal(I[clear], Io[clear])
    return float(err.max()) if err.size else 0.0


@pytest.mark.parametrize("m,excl", [(2, -1), (3, -1), (5, 0), (7, -1), (16, -1), (16, 0), (100, -1), (64, 700)])
def test_self_join_random_walk_exact(orc, m, excl):
    x = synth.random_walk(2600, np.random.default_rng(40 + m))
    check_self(orc, x, m, excl, exact_second=True)


@pytest.mark.parametrize("m", [64, 256])
def test_self_join_ecg_multi_tile(orc, m):
    x = synth.ecg_like(7000, np.random.default_rng(50 + m), n_anomalies=3)
    check_self(orc, x, m, -1)


def test_self_join_flat_and_nonfinite(orc):
    m = 32
    rng = np.random.default_rng(61)
    x = rng.standard_normal(4000)
    x[100:100 + m + 40] = 1.5      # 41 flat windows: flat partners outside the zone
    x[2000] = np.nan
    check_self(orc, x, m, -1, exact_second=True)
    y = rng.standard_normal(3000)
    y[700:700 + m + 10] = -2.0     # 11 flat windows, all inside each other's zone
    P, I, _ = gpu_self_join(y, m)
    assert np.allclose(P[700:711], np.sqrt(m)) and np.all(np.abs(I[700:711] - np.arange(700, 711)) > m // 2)
    check_self(orc, y, m, -1, exact_second=True)


def test_self_join_zone_covers_everything():
    x = np.random.default_rng(3).standard_normal(40)
    P, I, _ = gpu_self_join(x, 16, 24)  # W = 25: every other window is within 24
    assert np.all(np.isinf(P)) and np.all(I == -1)
    with pytest.raises(abjoin.AbjError):
        abjoin.self_join(dev(x), 16, 25)


def training_series(n, seed):
    return synth.ecg_like(n, np.random.default_rng(seed), n_anomalies=2)


def gpu_build(T, m, **kw):
    r = abjoin.dict_build(dev(T), m, **kw)
    torch.cuda.synchronize()
    r["dictionary"] = r["dictionary"].cpu().numpy()
    r["p_b"] = r["p_b"].cpu().numpy()
    return r


def replay(T, m, g, **kw):
    o = olearn.learn_dictionary(T, m, forced=list(g["chosen"]), tie_tol=2 * TOL, **kw)
    assert o["chosen"] == list(g["chosen"])
    assert o["segments"] == g["segments"]
    assert np.array_equal(o["bounds"], g["bounds"]) and np.array_equal(o["orig_start"], g["orig_start"])
    assert np.array_equal(o["dictionary"], g["dictionary"])
    fin = np.isfinite(o["p_b"])
    assert np.array_equal(fin, np.isfinite(g["p_b"]))
    assert np.abs(o["p_b"][fin] - g["p_b"][fin]).max() <= TOL
    if np.isfinite(o["e_max"]):
        assert abs(o["e_max"] - g["e_max"]) <= TOL, (o["e_max"], g["e_max"])
    else:
        assert o["e_max"] == g["e_max"] or (np.isnan(o["e_max"]) and np.isnan(g["e_max"]))
    return o


@pytest.mark.parametrize("m,value", [(128, 0.9), (64, 0.8)])
def test_dict_build_space_saving_lockstep(m, value):
    T = training_series(9000, 70 + m)
    print(f"[case] dict_build space_saving n={len(T)} m={m} s={value}", flush=True)
    g = gpu_build(T, m, stop="space_saving", value=value)
    assert len(g["chosen"]) > 3
    size = g["bounds"][-1]
    assert size >= (1 - value) * len(T)
    replay(T, m, g, stop="space_saving", value=value)


def test_dict_build_context_and_cap():
    T = training_series(5000, 81)
    m = 100
    g = gpu_build(T, m, context=2.5, stop="space_saving", value=0.0, max_iters=5)
    assert len(g["chosen"]) == 5
    assert all(b - a >= int(np.ceil(2.5 * m)) for a, b in g["segments"])
    replay(T, m, g, k=2.5, stop="space_saving", value=0.0, max_iters=5)


def test_dict_build_emax_stop():
    T = training_series(8000, 90)
    m = 128
    base = gpu_build(T, m, stop="space_saving", value=0.6)
    ch = list(base["chosen"])
    n = len(T)
    em = []
    for k in range(1, len(ch) + 1):
        segs = olearn.merge_elements([olearn.element_of(j, n, m, 1.5) for j in ch[:k]])
        em.append(olearn.e_max_of(T, segs, m))
    em = np.array(em)
    gaps = em[:-1] - em[1:]
    k = int(np.argmax(gaps)) + 1          # stop at step k (0-based) when target sits in this gap
    assert gaps[k - 1] > 4 * TOL, em
    target = 0.5 * (em[k - 1] + em[k])
    assert np.all(em[:k] > target)
    print(f"[case] dict_build e_max target={target:.4f} expected steps={k + 1}", flush=True)
    g = gpu_build(T, m, stop="e_max", value=target)
    assert list(g["chosen"]) == ch[:k + 1]
    assert g["e_max"] <= target + TOL
    replay(T, m, g, stop="e_max", value=target)


def test_dict_build_degenerate():
    m = 32
    T = np.random.default_rng(5).standard_normal(m + 5)   # W = 6 <= m/2: every P_B is +inf
    g = gpu_build(T, m)
    assert g["chosen"].size == 0 and g["segments"] == [] and np.isinf(g["e_max"]) and g["dictionary"].size == 0
    T = training_series(3000, 7)
    T[1500] = np.nan
    g = gpu_build(T, 64, stop="e_max", value=10.0, max_iters=3)   # NaN e_max never meets a target
    assert len(g["chosen"]) == 3 and np.isnan(g["e_max"])
    replay(T, 64, g, stop="e_max", value=10.0, max_iters=3)


def test_dict_build_rejects_bad_options():
    x = dev(training_series(2000, 1))
    for kw in (dict(context=0.0), dict(stop="space_saving", value=1.5), dict(stop="e_max", value=-1.0)):
        with pytest.raises(abjoin.AbjError) as e:
            abjoin.dict_build(x, 64, **kw)
        assert e.value.code == abjoin.ABJ_EINVAL


def test_dict_build_sized_buffers_and_source_index():
    # a run to exhaustion fits the buffers the sizing call asked for, and the
    # resident dictionary maps join results back to the training series
    T = training_series(3000, 12)
    m = 32
    print(f"[case] dict_build exhaustion n={len(T)} m={m}", flush=True)
    g = gpu_build(T, m, stop="space_saving", value=0.0)
    assert len(g["chosen"]) > 10
    replay(T, m, g, stop="space_saving", value=0.0)
    d = abjoin.Dictionary(dev(g["dictionary"]), g["bounds"], [m], orig_start=g["orig_start"])
    plain = abjoin.Dictionary(dev(g["dictionary"]), g["bounds"], [m])
    try:
        q = training_series(4000, 13)
        P, I = d.join(dev(q), m)
        src = d.source_index(I)
        same = plain.source_index(I)
        torch.cuda.synchronize()
        I, src, same = I.cpu().numpy(), src.cpu().numpy(), same.cpu().numpy()
        assert np.array_equal(same, I)
        ok = I >= 0
        assert ok.all()
        s = np.searchsorted(g["bounds"], I, side="right") - 1
        assert np.array_equal(src, g["orig_start"][s] + I - g["bounds"][s])
        for i in np.flatnonzero(ok)[:: max(1, ok.sum() // 200)]:
            assert np.array_equal(T[src[i]:src[i] + m], g["dictionary"][I[i]:I[i] + m])
        neg = torch.tensor([-1, len(g["dictionary"]), 0], dtype=torch.int64, device="cuda")
        assert d.source_index(neg).cpu().tolist() == [-1, -1, int(g["orig_start"][0])]
    finally:
        d.close()
        plain.close()
