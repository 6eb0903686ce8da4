"""FP64 CPU oracle for the AB-join matrix profile -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and its
Python binding) never imports, links or calls it, and the oracle shares no code
with that path: the C source here is compiled with gcc into its own shared
library, ``oracle/liborc.so``.

Each function follows a definition or algorithm of the paper (see the header of
``abjoin_oracle.c`` for the readings taken where the paper is silent):

* ``window_stats``  -- Def. 2/3 windows, mean and population deviation (two-pass)
* ``valid_windows`` -- Def. 8, windows that slide inside one dictionary segment
* ``ab_join``       -- Def. 7 matrix profile over the Def. 8 windows (Alg. 2)
* ``pair_dists``    -- Def. 4 z-normalised Euclidean distance for given pairs
* ``dist_matrix``   -- every pairwise distance (tiny inputs only)
* ``self_join``     -- Alg. 1's self-join (P_B), intra-similarity join with exclusion zone
* ``dist_profile``  -- Def. 4 distance profile (Alg. 1's profile of the chosen window)
* ``ab_join_stream`` -- the same join as ``ab_join`` by an independently written
  FP64 diagonal sweep with O(1) work per pair (``stream_oracle.c``), for joins
  too large for the brute force (a held-out series against a whole database)
* ``learn_dictionary`` (in ``oracle.learn``) -- Alg. 1
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "abjoin_oracle.c")
_SRC_STREAM = os.path.join(_HERE, "stream_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, _SRC_STREAM,
               "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                      os.path.getmtime(_SRC_STREAM)):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_window_stats.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int32, _f64p, _f64p, _u8p, _u8p]
        lib.orc_valid_windows.argtypes = [_i64p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _u8p]
        lib.orc_ab_join.argtypes = [
            _f64p, ctypes.c_int64, _f64p, ctypes.c_int64, _i64p, ctypes.c_int32, ctypes.c_int32,
            _i64p, ctypes.c_int64, _f64p, _i64p, _f64p, ctypes.c_int32,
        ]
        lib.orc_pair_dists.argtypes = [
            _f64p, ctypes.c_int64, _f64p, ctypes.c_int64, ctypes.c_int32, _i64p, _i64p, ctypes.c_int64, _f64p,
        ]
        lib.orc_dist_matrix.argtypes = [_f64p, ctypes.c_int64, _f64p, ctypes.c_int64, ctypes.c_int32, _f64p]
        lib.orc_self_join.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, _f64p, _i64p,
                                      ctypes.c_int32]
        lib.orc_dist_profile.argtypes = [_f64p, ctypes.c_int64, ctypes.c_int32, _f64p, _f64p]
        lib.orc_ab_join_stream.argtypes = [_f64p, ctypes.c_int64, _f64p, ctypes.c_int64, _i64p, ctypes.c_int32,
                                           ctypes.c_int32, _f64p, _i64p, ctypes.c_int32]
        for f in ("orc_window_stats", "orc_valid_windows", "orc_ab_join", "orc_pair_dists", "orc_dist_matrix",
                  "orc_self_join", "orc_dist_profile", "orc_ab_join_stream"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _i64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def _p(a, t):
    return a.ctypes.data_as(t)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def window_stats(x, m):
    """(mu, sd, flat, bad) for every length-m window of x."""
    x = _f64(x)
    W = len(x) - m + 1
    mu, sd = np.empty(W), np.empty(W)
    flat, bad = np.empty(W, np.uint8), np.empty(W, np.uint8)
    _check(_load().orc_window_stats(_p(x, _f64p), len(x), m, _p(mu, _f64p), _p(sd, _f64p), _p(flat, _u8p),
                                    _p(bad, _u8p)), "window_stats")
    return mu, sd, flat.astype(bool), bad.astype(bool)


def valid_windows(bounds, n, m):
    bounds = _i64(bounds)
    out = np.empty(n - m + 1, np.uint8)
    _check(_load().orc_valid_windows(_p(bounds, _i64p), len(bounds) - 1, n, m, _p(out, _u8p)), "valid_windows")
    return out.astype(bool)


def ab_join(query, dictionary, bounds, m, rows=None, threads=0, second=False):
    """Brute-force FP64 AB-join of ``query`` against the Def. 8 windows of ``dictionary``.

    Returns (P, I) or (P, I, P2) with ``second=True`` (P2 = best distance over the
    other reference windows).  ``rows`` restricts the evaluation to those query
    windows (results in the order given).
    """
    q, d, b = _f64(query), _f64(dictionary), _i64(bounds)
    if rows is None:
        nrows = len(q) - m + 1
        rp = None
    else:
        rows = _i64(rows)
        nrows = len(rows)
        rp = _p(rows, _i64p)
    P, I = np.empty(max(nrows, 0)), np.empty(max(nrows, 0), np.int64)
    P2 = np.empty(max(nrows, 0))
    _check(_load().orc_ab_join(_p(q, _f64p), len(q), _p(d, _f64p), len(d), _p(b, _i64p), len(b) - 1, m,
                               rp, nrows, _p(P, _f64p), _p(I, _i64p), _p(P2, _f64p), int(threads)), "ab_join")
    return (P, I, P2) if second else (P, I)


def pair_dists(query, ref, m, ii, jj):
    q, d, ii, jj = _f64(query), _f64(ref), _i64(ii), _i64(jj)
    out = np.empty(len(ii))
    _check(_load().orc_pair_dists(_p(q, _f64p), len(q), _p(d, _f64p), len(d), m, _p(ii, _i64p), _p(jj, _i64p),
                                  len(ii), _p(out, _f64p)), "pair_dists")
    return out


def dist_matrix(query, ref, m):
    q, d = _f64(query), _f64(ref)
    D = np.empty((len(q) - m + 1, len(d) - m + 1))
    _check(_load().orc_dist_matrix(_p(q, _f64p), len(q), _p(d, _f64p), len(d), m, _p(D, _f64p)), "dist_matrix")
    return D


def self_join(x, m, excl=None, threads=0):
    """Self-join matrix profile with exclusion |i - j| <= excl (default floor(m/2))."""
    x = _f64(x)
    excl = m // 2 if excl is None else int(excl)
    W = len(x) - m + 1
    P, I = np.empty(W), np.empty(W, np.int64)
    _check(_load().orc_self_join(_p(x, _f64p), len(x), m, excl, _p(P, _f64p), _p(I, _i64p), int(threads)),
           "self_join")
    return P, I


def dist_profile(x, m, w):
    x, w = _f64(x), _f64(w)
    S = np.empty(len(x) - m + 1)
    _check(_load().orc_dist_profile(_p(x, _f64p), len(x), m, _p(w, _f64p), _p(S, _f64p)), "dist_profile")
    return S


def ab_join_stream(query, dictionary, bounds, m, threads=0):
    """The AB-join of ``ab_join`` by the streaming oracle: (P, I) for every query window.

    Same definition and conventions; an FP64 diagonal sweep (O(1) per pair,
    exact restarts every 256 steps) picks each row's column and its distance is
    then recomputed directly.  Pinned against the brute force by the tests."""
    q, d, b = _f64(query), _f64(dictionary), _i64(bounds)
    W = len(q) - m + 1
    P, I = np.empty(max(W, 0)), np.empty(max(W, 0), np.int64)
    _check(_load().orc_ab_join_stream(_p(q, _f64p), len(q), _p(d, _f64p), len(d), _p(b, _i64p), len(b) - 1, m,
                                      _p(P, _f64p), _p(I, _i64p), int(threads)), "ab_join_stream")
    return P, I
