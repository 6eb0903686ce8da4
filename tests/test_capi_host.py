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
