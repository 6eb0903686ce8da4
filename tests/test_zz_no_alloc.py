"""ab_join_noalloc (the AB-join with a fixed library-held workspace, for callers
that cannot allocate) against ab_join, through the C-ABI: equal results on two
calls in a row, the second with a smaller input, for the FP32 tier with
per-chunk keys, with the atomic merge (a join whose per-chunk keys would not
fit the workspace) and for a 16-bit tier; a join too large for the workspace
is rejected before anything is written."""
import ctypes

import numpy as np
import pytest
import torch

import _parity
from paper_2112_12965_amd import abjoin, synth

pytestmark = pytest.mark.gpu


def call(fn, q, d, bounds, m, tier="fp32", fill=None):
    b = np.ascontiguousarray(bounds, dtype=np.int64)
    W = q.numel() - m + 1
    P = torch.empty(W, dtype=torch.float32, device="cuda")
    I = torch.empty(W, dtype=torch.int64, device="cuda")
    if fill is not None:
        P.fill_(fill)
        I.fill_(-7)
    o = abjoin.abj_opts(abjoin.TIERS[tier], 0, 0, 0)
    rc = getattr(abjoin.lib(), fn)(q.data_ptr(), q.numel(), d.data_ptr(), d.numel(),
                                   b.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(b) - 1, m, P.data_ptr(),
                                   I.data_ptr(), ctypes.byref(o), None)
    return rc, P, I


def both(q, d, bounds, m, tier="fp32"):
    print(f"[case] noalloc vs ab_join tier={tier} n_q={q.numel()} n_d={d.numel()} m={m}", flush=True)
    rc0, P0, I0 = call("ab_join", q, d, bounds, m, tier)
    assert rc0 == abjoin.ABJ_OK, abjoin.last_error()
    rc1, P1, I1 = call("ab_join_noalloc", q, d, bounds, m, tier)
    assert rc1 == abjoin.ABJ_OK, abjoin.last_error()
    torch.cuda.synchronize()
    assert torch.equal(P0, P1) and torch.equal(I0, I1)
    return P1.cpu().numpy(), I1.cpu().numpy()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.mark.parametrize("tier", ["fp32", "bf16"])
def test_noalloc_equals_ab_join_two_calls(orc, tier):
    rng = np.random.default_rng(77)
    q_big, d_big = synth.ecg_like(40000, rng, n_anomalies=3), synth.ecg_like(12000, rng)
    b_big = [0, 3000, 3100, 7000, 12000]
    q_small, d_small = synth.random_walk(3000, rng), synth.random_walk(2500, rng)
    b_small = [0, 1300, 2500]
    for q, d, b, m in ((q_big, d_big, b_big, 128), (q_small, d_small, b_small, 64)):
        P, I = both(dev(q), dev(d), b, m, tier)
        rows = np.unique(np.concatenate([rng.choice(len(P), 200, replace=False), [0, len(P) - 1]]))
        Po, Io, P2o = orc.ab_join(q, d, b, m, rows=rows, second=True)
        _parity.compare(P[rows], I[rows], Po, Io, P2o, 1e-3, orc, q, d, m, b, rows=rows)


def test_noalloc_atomic_merge_then_small(orc):
    # 200k query windows x 64 chunks of keys (about 100 MB) do not fit the
    # workspace, so the tiles merge by atomics; the second call is small again
    rng = np.random.default_rng(78)
    q, d = dev(synth.random_walk(200_000, rng)), dev(synth.random_walk(65_000, rng))
    both(q, d, [0, 65_000], 100)
    q2, d2 = dev(synth.random_walk(5000, rng)), dev(synth.random_walk(4000, rng))
    both(q2, d2, [0, 4000], 100)


def test_noalloc_rejects_oversized_join_without_writing():
    rng = np.random.default_rng(79)
    q = dev(synth.random_walk(800_000, rng))
    d = dev(synth.random_walk(1000, rng))
    rc, P, I = call("ab_join_noalloc", q, d, [0, 1000], 64, fill=3.5)
    assert rc == abjoin.ABJ_EINVAL and "workspace" in abjoin.last_error()
    torch.cuda.synchronize()
    assert torch.all(P == 3.5) and torch.all(I == -7)
    # a normal call still works afterwards
    q2, d2 = dev(synth.random_walk(3000, rng)), dev(synth.random_walk(3000, rng))
    both(q2, d2, [0, 3000], 64)
