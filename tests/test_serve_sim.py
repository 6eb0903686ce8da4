"""Scheduler tests of the serving loop on the host-simulation backend (no GPU).

The simulation backend runs the library's real scheduler (admission by slots
and memory, FIFO order, continuous batching with two launches in flight,
cancellation, statistics) but replaces the GPU work by a wait of
pairs / rate seconds and a deterministic fake result.
"""
import time

import numpy as np
import pytest

from paper_2112_12965_amd import abjoin


def make(**kw):
    base = dict(backend="sim", sim_ms=(64, 128, 256), sim_dict_windows=60000, sim_pairs_per_s=5e11,
                max_slots=64, mem_budget=8 << 30)
    base.update(kw)
    return abjoin.Server(**base)


def run_all(srv, reqs):
    ids = [srv.submit(q, m) for q, m in reqs]
    for i in ids:
        assert srv.wait(i, 20000) == abjoin.ABJ_OK
    return ids, [srv.result(i) for i in ids]


def test_results_and_timestamps():
    srv = make()
    rng = np.random.default_rng(0)
    reqs = [(rng.standard_normal(int(n)), m) for n, m in zip(rng.integers(1024, 8192, 12), [64, 128, 256] * 4)]
    ids, res = run_all(srv, reqs)
    for rid, (q, m), (P, I, st) in zip(ids, reqs, res):
        W = len(q) - m + 1
        assert P.shape == (W,) and I.shape == (W,)
        i = np.arange(W)
        np.testing.assert_allclose(P, ((i * 7 + rid) % 100) * 0.1, rtol=1e-6)
        assert st["t_arrive"] <= st["t_admit"] <= st["t_start"] <= st["t_device_done"] <= st["t_done"]
        assert st["pairs"] == W * 60000 and st["status"] == 0
    s = srv.stats()
    assert s["submitted"] == 12 and s["completed"] == 12 and s["pairs"] == sum(r[2]["pairs"] for r in res)
    assert 0 < s["p50_s"] <= s["p99_s"] <= s["max_s"]
    srv.close()


def _max_overlap(stats):
    # slots and memory are held from admission until the device has finished
    ev = sorted([(s["t_admit"], 1) for s in stats] + [(s["t_device_done"], -1) for s in stats],
                key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_memory_budget_limits_concurrency():
    # budget for two requests of this size at a time
    probe = make()
    rid = probe.submit(np.zeros(20000), 128)
    probe.wait(rid)
    probe.close()
    srv = make(mem_budget=2 * 20000 * 8 * 12, sim_pairs_per_s=2e11)
    reqs = [(np.zeros(20000), 128)] * 6
    _, res = run_all(srv, reqs)
    assert _max_overlap([r[2] for r in res]) <= 2
    srv.close()


def test_single_slot_is_sequential_and_fifo():
    srv = make(max_slots=1)
    reqs = [(np.zeros(4096), 64)] * 5
    _, res = run_all(srv, reqs)
    st = [r[2] for r in res]
    for a, b in zip(st, st[1:]):
        assert b["t_admit"] >= a["t_device_done"] - 1e-9  # admitted only after the previous one finished
        assert b["t_admit"] >= a["t_admit"]        # in submission order
    srv.close()


def test_continuous_batching_launches_while_busy():
    srv = make(sim_pairs_per_s=1e11)
    a = srv.submit(np.zeros(60000), 64)  # ~36 ms of simulated work
    time.sleep(0.005)
    b = srv.submit(np.zeros(2000), 64)
    assert srv.wait(a, 20000) == 0 and srv.wait(b, 20000) == 0
    sa, sb = srv.result(a)[2], srv.result(b)[2]
    assert sb["batch"] == sa["batch"] + 1
    assert sb["t_start"] < sa["t_device_done"]  # launched while the first launch was still running
    srv.close()


def test_cancel_queued_request():
    srv = make(max_slots=1, sim_pairs_per_s=2e10)
    ids = [srv.submit(np.zeros(8192), 128) for _ in range(4)]
    assert srv.cancel(ids[3]) == abjoin.ABJ_OK
    assert srv.wait(ids[3], 1000) == abjoin.ABJ_ECANCELED
    with pytest.raises(abjoin.AbjError) as e:
        srv.result(ids[3])
    assert e.value.code == abjoin.ABJ_ECANCELED
    for i in ids[:3]:
        assert srv.wait(i, 20000) == abjoin.ABJ_OK
    assert srv.cancel(ids[0]) == abjoin.ABJ_EBUSY  # finished requests are not cancelable
    assert srv.stats()["canceled"] == 1
    srv.close()


def test_invalid_requests_rejected_without_disturbing_others():
    srv = make(mem_budget=1 << 22)
    good = srv.submit(np.zeros(3000), 128)
    for q, m, code in [(np.zeros(100), 128, abjoin.ABJ_EINVAL),   # shorter than m
                       (np.zeros(3000), 100, abjoin.ABJ_EINVAL),  # m not a dictionary window length
                       (np.zeros(1 << 20), 64, abjoin.ABJ_ENOMEM)]:  # larger than the whole budget
        with pytest.raises(abjoin.AbjError) as e:
            srv.submit(q, m)
        assert e.value.code == code
    assert srv.wait(good, 20000) == abjoin.ABJ_OK
    s = srv.stats()
    assert s["rejected"] == 3 and s["completed"] == 1
    assert srv.wait(12345, 0) == abjoin.ABJ_ENOTFOUND
    srv.close()


def test_drain_and_destroy_with_pending_requests():
    srv = make(max_slots=1, sim_pairs_per_s=1e11)
    ids = [srv.submit(np.zeros(4096), 64) for _ in range(20)]
    assert srv.drain(20000) == abjoin.ABJ_OK
    assert srv.stats()["completed"] == 20
    more = [srv.submit(np.zeros(60000), 64) for _ in range(10)]
    srv.close()  # cancels what is still queued; must not hang


def test_copied_and_borrowed_submissions():
    srv = make()
    rng = np.random.default_rng(3)
    qs = [rng.standard_normal(int(n)) for n in rng.integers(1024, 4096, 8)]
    ids = [srv.submit(q, 64, copy=(k % 2 == 0)) for k, q in enumerate(qs)]
    for i in ids:
        assert srv.wait(i, 20000) == abjoin.ABJ_OK
    for rid, q in zip(ids, qs):
        P, I, st = srv.result(rid)
        W = len(q) - 63
        assert P.shape == (W,) and I.shape == (W,) and st["status"] == 0
        np.testing.assert_allclose(P, ((np.arange(W) * 7 + rid) % 100) * 0.1, rtol=1e-6)
    assert not srv._reqs  # borrowed buffers are released with the result
    with pytest.raises(abjoin.AbjError) as e:
        srv.submit(np.zeros(10), 64)
    assert e.value.code == abjoin.ABJ_EINVAL
    srv.close()


def test_batch_takes_half_the_slots():
    srv = make(max_slots=8, sim_pairs_per_s=2e11)
    ids = [srv.submit(np.zeros(4096), 64) for _ in range(24)]
    assert srv.drain(60000) == abjoin.ABJ_OK
    per_batch = {}
    for i in ids:
        b = srv.result(i)[2]["batch"]
        per_batch[b] = per_batch.get(b, 0) + 1
    assert max(per_batch.values()) <= 4 and len(per_batch) >= 6
    srv.close()
