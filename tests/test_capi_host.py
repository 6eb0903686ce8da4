"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function its header declares, and rejects invalid arguments before
touching the GPU."""
import ctypes

import numpy as np
import pytest

from paper_2112_12965_amd import abjoin


@pytest.fixture(scope="module")
def L():
    return abjoin.lib()


def test_exports_every_declared_symbol(L):
    names = abjoin.header_functions()
    assert {"ab_join", "abj_version", "abj_last_error", "abj_init", "abj_window_stats"} <= set(names)
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/abjoin.h but not exported"


def test_version(L):
    v = L.abj_version()
    assert v >= 1


def _call_join(L, m=16, nq=100, nd=100, bounds=(0, 100), tier=0, refine_k=0, flags=0):
    b = np.asarray(bounds, dtype=np.int64)
    o = abjoin.abj_opts(tier, refine_k, flags, 0)
    return L.ab_join(None, nq, None, nd, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(b) - 1, m,
                     None, None, ctypes.byref(o), None)


@pytest.mark.parametrize("kw", [
    dict(m=1), dict(m=0), dict(m=5000), dict(nq=10, m=16), dict(nd=0, bounds=(0, 0)),
    dict(bounds=(0, 50, 50, 100)), dict(bounds=(1, 100)), dict(bounds=(0, 99)),
    dict(tier=7), dict(refine_k=9), dict(refine_k=-1), dict(flags=1),
])
def test_invalid_arguments_rejected_before_any_gpu_work(L, kw):
    assert _call_join(L, **kw) == abjoin.ABJ_EINVAL
    assert abjoin.last_error()


def test_null_device_pointers_rejected(L):
    assert _call_join(L) == abjoin.ABJ_EINVAL
    assert "NULL" in abjoin.last_error()


def test_window_stats_rejects_bad_m(L):
    assert L.abj_window_stats(None, 10, 1, None, None, None, None) == abjoin.ABJ_EINVAL
    assert L.abj_window_stats(None, 10, 11, None, None, None, None) == abjoin.ABJ_EINVAL


def _sizing(L, n, m, context=1.5, stop=0, value=0.9, max_iters=0, outs=(True, True, True)):
    o = abjoin.abj_learn_opts(context, value, stop, max_iters)
    ns, nc, nd = ctypes.c_int32(-7), ctypes.c_int32(-7), ctypes.c_int64(-7)
    rc = L.dict_build(None, n, m, ctypes.byref(o), None, 0, ctypes.byref(ns) if outs[0] else None, None, 0,
                      ctypes.byref(nc) if outs[1] else None, None, ctypes.byref(nd) if outs[2] else None, None,
                      None, None)
    return rc, ns.value, nc.value, nd.value


def test_dict_build_sizing_call_needs_no_series_and_no_gpu(L):
    # n = 1000, m = 16: windows are more than 8 apart, so at most
    # ceil(985 / 9) = 110 are chosen; segments hold at least ceil(1.5 * 16) = 24
    # samples and do not touch, so at most 1000 // 25 + 1 = 41 of them
    assert _sizing(L, 1000, 16) == (abjoin.ABJ_OK, 41, 110, 1000)
    assert _sizing(L, 1000, 16, max_iters=5) == (abjoin.ABJ_OK, 5, 5, 1000)
    rc, ns, nc, nd = _sizing(L, 1000, 16, outs=(False, True, False))
    assert rc == abjoin.ABJ_OK and (ns, nc, nd) == (-7, 110, -7)


@pytest.mark.parametrize("kw", [dict(m=1), dict(m=5000), dict(n=10, m=16), dict(context=0.0), dict(stop=9),
                                dict(value=2.0), dict(max_iters=-1), dict(outs=(False, False, False))])
def test_dict_build_sizing_call_rejects_bad_arguments(L, kw):
    args = dict(n=1000, m=16)
    args.update(kw)
    assert _sizing(L, **args)[0] == abjoin.ABJ_EINVAL
    assert abjoin.last_error()


def test_dict_build_real_call_still_needs_the_series(L):
    o = abjoin.abj_learn_opts(1.5, 0.9, 0, 0)
    segs = np.zeros(8, dtype=np.int64)
    ns = ctypes.c_int32(0)
    assert L.dict_build(None, 1000, 16, ctypes.byref(o), segs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 4,
                        ctypes.byref(ns), None, 0, None, None, None, None, None, None) == abjoin.ABJ_EINVAL


@pytest.mark.parametrize("seed,m,context", [(0, 4, 1.5), (1, 8, 1.5), (2, 16, 1.0), (3, 6, 3.0), (4, 10, 1.2)])
def test_dict_build_sizing_bounds_hold_for_a_run_to_exhaustion(L, seed, m, context):
    # Alg. 1 run by the oracle until nothing is left to choose (space saving 0):
    # the most segments, choices and samples any run can produce
    from oracle import learn as orl

    rng = np.random.default_rng(seed)
    n = int(rng.integers(3 * m, 240))
    T = np.cumsum(rng.standard_normal(n))
    r = orl.learn_dictionary(T, m, k=context, stop="space_saving", value=0.0)
    rc, ns, nc, nd = _sizing(L, n, m, context=context, value=0.0)
    assert rc == abjoin.ABJ_OK
    assert len(r["segments"]) <= ns and len(r["chosen"]) <= nc and len(r["dictionary"]) <= nd


def test_dict_create_rejects_a_negative_orig_start_before_any_gpu_work(L):
    d = np.zeros(100)
    b = np.array([0, 50, 100], dtype=np.int64)
    orig = np.array([0, -3], dtype=np.int64)
    ms = (ctypes.c_int32 * 1)(16)
    h = ctypes.c_void_p()
    assert L.abj_dict_create(d.ctypes.data, 100, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 2,
                             orig.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ms, 1,
                             ctypes.byref(h)) == abjoin.ABJ_EINVAL
    assert "orig_start" in abjoin.last_error() and not h.value


def test_source_index_rejects_a_null_dictionary(L):
    assert L.abj_dict_source_index(None, None, 4, None, None) == abjoin.ABJ_EINVAL
