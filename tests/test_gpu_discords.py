"""GPU parity of discord discovery.

* topk_discords equals the oracle's greedy exactly on float profiles with
  ties, NaN and inf (same values, same tie rule);
* discords (exact top-K from the dictionary join) equals the oracle's top-K on
  the exact FP64 join against the reference: same rows, values within the
  FP32 bar, neighbours valid; it must join fewer rows than the whole query
  where the dictionary is good, and its certification bits must agree with
  the oracle's tests on the same P_hat and e_max.
"""
import numpy as np
import pytest
import torch

from oracle import discords as odisc
from paper_2112_12965_amd import abjoin

pytestmark = pytest.mark.gpu
TOL = 1e-3


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.mark.parametrize("seed", range(6))
def test_topk_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    W = int(rng.integers(1, 5000))
    P = np.round(rng.uniform(0, 5, W), 1).astype(np.float32)
    P[rng.random(W) < 0.05] = np.nan
    P[rng.random(W) < 0.02] = np.inf
    P[rng.random(W) < 0.02] = -np.inf
    K, excl = int(rng.integers(1, 40)), int(rng.integers(0, 50))
    rows, vals = abjoin.topk_discords(dev(P, torch.float32), K, excl)
    ro, vo = odisc.topk_discords(P.astype(np.float64), K, excl)
    assert np.array_equal(rows, ro) and np.array_equal(vals.astype(np.float64), vo)


def periodic(n, rng, bursts=(), amp=0.15):
    t = np.arange(n) + rng.uniform(0, 1000)
    x = np.sin(2 * np.pi * t / 100) + 0.4 * np.sin(2 * np.pi * t / 37) + rng.normal(0, 0.02, n)
    for b in bursts:
        x[b:b + 60] += np.cumsum(rng.normal(0, amp, 60))
    return x


def run_case(orc, q, ref, bounds, m, K, space_saving, amp_note=""):
    print(f"[case] discords n_q={len(q)} n_ref={len(ref)} m={m} K={K} s={space_saving} {amp_note}", flush=True)
    # learning phase (on the first segment of the reference) and dictionary join on the GPU;
    # the dictionary's windows are windows of the reference, so P_hat bounds P from above
    g = abjoin.dict_build(dev(ref[:bounds[1]]), m, stop="space_saving", value=space_saving)
    Ph, _ = abjoin.ab_join(dev(q), g["dictionary"], g["bounds"], m)
    em = g["e_max"]
    r = abjoin.discords(dev(q), Ph, em, dev(ref), bounds, m, K)
    torch.cuda.synchronize()
    ro, vo, io = odisc.exact_discords(q, ref, bounds, m, K)
    print("gpu", r["rows"], r["values"], r["rows_exact"], r["rounds"], r["certified"], "oracle", ro, vo, flush=True)
    assert np.array_equal(r["rows"], ro)
    assert np.abs(r["values"].astype(np.float64) - vo).max() <= TOL
    d = orc.pair_dists(q, ref, m, ro, r["neighbors"])
    assert np.all(d - vo <= TOL)
    Phh = Ph.cpu().numpy().astype(np.float64)
    want = int(odisc.top_certified(Phh, em)) | (int(odisc.top_certified(Phh, em, m - 1)) << 1)
    assert r["certified"] == want
    return r, len(q) - m + 1


@pytest.mark.parametrize("seed", range(3))
def test_exact_discords_from_dictionary(orc, seed):
    rng = np.random.default_rng(seed)
    m = 128
    ref = periodic(6000, rng)
    q = periodic(20000, rng, [3000, 9000, 15000])
    r, W = run_case(orc, q, ref, [0, len(ref)], m, 3, 0.5)
    assert r["rows_exact"] < W  # the bound spared part of the query


def test_top_discord_certified_case(orc):
    rng = np.random.default_rng(1)
    m = 100
    ref = periodic(4000, rng)
    q = periodic(8000, rng, [5000], amp=0.5)
    r, W = run_case(orc, q, ref, [0, len(ref)], m, 1, 0.3, "strong burst")
    assert r["certified"] & 2 and r["rounds"] == 1 and r["rows_exact"] <= 3 * 1024


def test_many_discords_and_segmented_reference(orc):
    rng = np.random.default_rng(9)
    m = 64
    ref = periodic(9000, rng)
    bounds = [0, 3000, 6000, 9000]
    q = periodic(12000, rng, [1000, 4000, 8000, 11000], amp=0.3)
    run_case(orc, q, ref, bounds, m, 8, 0.6)


def test_no_bound_and_no_dictionary_window(orc):
    rng = np.random.default_rng(4)
    m = 64
    ref = periodic(3000, rng)
    q = periodic(5000, rng, [2500])
    # P_hat = +inf everywhere (a dictionary without a window): every row is joined
    Ph = torch.full((len(q) - m + 1,), float("inf"), dtype=torch.float32, device="cuda")
    r = abjoin.discords(dev(q), Ph, -1.0, dev(ref), [0, len(ref)], m, 2)
    ro, vo, _ = odisc.exact_discords(q, ref, [0, len(ref)], m, 2)
    assert np.array_equal(r["rows"], ro) and r["rows_exact"] == len(q) - m + 1 and r["certified"] == 0
    with pytest.raises(abjoin.AbjError):
        abjoin.discords(dev(q), Ph, float("nan"), dev(ref), [0, len(ref)], m, 2)
