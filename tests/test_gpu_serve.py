"""GPU tests of the resident dictionary and the continuous-batching server.

* ab_join_dict equals ab_join on the same inputs (bitwise);
* every served result (query copied or borrowed) equals the same request
  joined alone through the resident dictionary (bitwise: a request's tiles and
  arithmetic do not depend on what else shares its launch), under mixed query
  lengths and window lengths, with queueing forced by slot and memory limits;
* served results meet the FP32 parity bar against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import _parity
from paper_2112_12965_amd import abjoin, synth

pytestmark = pytest.mark.gpu
MS = (64, 128, 256)


@pytest.fixture(scope="module")
def served_dict():
    w = synth.WORKLOADS["serve_dict64x1000"]()
    d = abjoin.Dictionary(w["dict"], w["bounds"], MS)
    yield w, d
    d.close()


def requests(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        L = int(np.exp(rng.uniform(np.log(1024), np.log(16384))))
        out.append((synth.ecg_like(L, rng, n_anomalies=1 if L > 4000 else 0), MS[k % 3]))
    return out


@pytest.mark.parametrize("tier", ["fp32", "bf16"])
def test_dict_join_equals_one_shot(served_dict, tier):
    w, d = served_dict
    q = synth.ecg_like(9000, np.random.default_rng(1))
    qd, dd = torch.from_numpy(q).cuda(), torch.from_numpy(w["dict"]).cuda()
    for m in MS:
        P1, I1 = d.join(qd, m, tier=tier)
        P2, I2 = abjoin.ab_join(qd, dd, w["bounds"], m, tier=tier)
        torch.cuda.synchronize()
        assert torch.equal(P1, P2) and torch.equal(I1, I2), m


def alone(d, q, m, tier):
    P, I = d.join(torch.from_numpy(q).cuda(), m, tier=tier)
    torch.cuda.synchronize()
    return P.cpu().numpy(), I.cpu().numpy()


@pytest.mark.parametrize("tier,slots,budget,copy", [("fp32", 64, 8 << 30, False), ("fp32", 64, 8 << 30, True),
                                                    ("fp32", 3, 8 << 30, False), ("fp32", 64, 24 << 20, False),
                                                    ("bf16", 8, 8 << 30, False), ("bf16", 8, 8 << 30, True)])
def test_served_equals_alone(served_dict, tier, slots, budget, copy):
    w, d = served_dict
    reqs = requests(24, seed=7)
    print(f"[case] server tier={tier} slots={slots} budget={budget} copy={copy}", flush=True)
    srv = abjoin.Server(d, tier=tier, max_slots=slots, mem_budget=budget)
    ids = [srv.submit(q, m, copy=copy) for q, m in reqs]
    res = []
    for i in ids:
        assert srv.wait(i, 60000) == abjoin.ABJ_OK, abjoin.last_error()
        res.append(srv.result(i))
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs)
    batches = {r[2]["batch"] for r in res}
    if slots < 64 or budget < (1 << 30):
        assert len(batches) > 1  # the limits forced several launches
    for (q, m), (P, I, rs) in zip(reqs, res):
        Pa, Ia = alone(d, q, m, tier)
        assert np.array_equal(P, Pa) and np.array_equal(I, Ia)
        assert rs["t_arrive"] <= rs["t_admit"] <= rs["t_start"] <= rs["t_device_done"] <= rs["t_done"]


def test_served_results_match_oracle(served_dict, orc):
    w, d = served_dict
    reqs = requests(6, seed=11)
    srv = abjoin.Server(d, tier="fp32", max_slots=4)
    ids = [srv.submit(q, m) for q, m in reqs]
    for (q, m), i in zip(reqs, ids):
        assert srv.wait(i, 60000) == abjoin.ABJ_OK
        P, I, _ = srv.result(i)
        Po, Io, P2o = orc.ab_join(q, w["dict"], w["bounds"], m, second=True)
        _parity.compare(P, I, Po, Io, P2o, 1e-3, orc, q, w["dict"], m, w["bounds"])
    srv.close()


def test_cancel_and_reject_on_gpu(served_dict):
    w, d = served_dict
    srv = abjoin.Server(d, tier="fp32", max_slots=1)
    ids = [srv.submit(synth.ecg_like(16000, np.random.default_rng(k)), 256) for k in range(6)]
    assert srv.cancel(ids[-1]) in (abjoin.ABJ_OK, abjoin.ABJ_EBUSY)
    with pytest.raises(abjoin.AbjError):
        srv.submit(np.zeros(10), 64)
    for i in ids[:-1]:
        assert srv.wait(i, 60000) == abjoin.ABJ_OK
    assert srv.drain(60000) == abjoin.ABJ_OK
    srv.close()


def test_serving_workload_sample_equals_alone(served_dict):
    """The serving workload's request mix at scale (1,024 requests, lengths
    log-uniform 1,024-65,536, m in {64, 128, 256}) submitted at once: 48 sampled
    requests are bitwise equal to the same joins run alone."""
    w, d = served_dict
    sched = synth.serving_schedule(1024, 1e9, synth.rng_for(4, 0))
    pool = synth.ecg_like(1 << 21, synth.rng_for(3, 0))
    offs = synth.rng_for(4, 99).integers(0, len(pool) - 65536, len(sched))
    print("[case] serving mix 1024 requests", flush=True)
    srv = abjoin.Server(d, tier="fp32", max_slots=512, mem_budget=2 << 30)
    qs = [pool[o:o + r.length] for o, r in zip(offs, sched)]
    ids = [srv.submit(q, r.m) for q, r in zip(qs, sched)]
    assert srv.drain(120000) == abjoin.ABJ_OK
    st = srv.stats()
    assert st["completed"] == len(sched) and st["batches"] > 1
    pick = set(np.random.default_rng(0).choice(len(sched), 48, replace=False).tolist())
    for k, i in enumerate(ids):
        P, I, _ = srv.result(i)
        if k in pick:
            Pa, Ia = alone(d, qs[k], sched[k].m, "fp32")
            assert np.array_equal(P, Pa) and np.array_equal(I, Ia), k
    srv.close()


def test_short_windows_served_and_resident(orc):
    # the FP32 engine's exact path for windows shorter than 8 samples, through
    # the resident dictionary and a serving batch that mixes it with m = 64
    rng = np.random.default_rng(21)
    dct = rng.standard_normal(3000)
    bounds = [0, 1000, 2200, 3000]
    d = abjoin.Dictionary(dct, bounds, (3, 64))
    try:
        reqs = [(rng.standard_normal(int(rng.integers(800, 4000))), (3, 64)[k % 2]) for k in range(6)]
        print("[case] short windows served", flush=True)
        srv = abjoin.Server(d, tier="fp32", max_slots=8)
        ids = [srv.submit(q, m) for q, m in reqs]
        for (q, m), i in zip(reqs, ids):
            assert srv.wait(i, 60000) == abjoin.ABJ_OK
            P, I, _ = srv.result(i)
            Pa, Ia = alone(d, q, m, "fp32")
            assert np.array_equal(P, Pa) and np.array_equal(I, Ia)
            if m == 3:
                Po, Io, P2o = orc.ab_join(q, dct, bounds, m, second=True)
                _parity.compare(P, I, Po, Io, P2o, 1e-3, orc, q, dct, m, bounds)
        srv.close()
    finally:
        d.close()
