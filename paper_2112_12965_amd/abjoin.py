"""ctypes binding of libabjoin.so (argument marshalling only).

Every computation happens in the HIP library; this module only turns PyTorch
CUDA tensors into device pointers and the current HIP stream into the stream
argument, and maps non-OK status codes to exceptions.  If the library has not
been built the first call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabjoin.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "abjoin.h")

ABJ_FLAG_NO_REFINE, ABJ_FLAG_PEARSON = 1, 2
ABJ_OK, ABJ_EINVAL, ABJ_ENOMEM, ABJ_EHIP, ABJ_EBUSY, ABJ_ECANCELED, ABJ_ETIMEOUT, ABJ_ENOTFOUND = (
    0, -1, -2, -3, -4, -5, -6, -7)
TIERS = {"fp32": 0, "bf16": 1, "fp16": 2}
FLAG_FLAT, FLAG_BAD = 1, 2

_lib = None


class AbjError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"abjoin error {code}: {msg}")
        self.code = code


class abj_opts(ctypes.Structure):
    _fields_ = [("tier", ctypes.c_int32), ("refine_k", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class abj_learn_opts(ctypes.Structure):
    _fields_ = [("context", ctypes.c_double), ("stop_value", ctypes.c_double), ("stop", ctypes.c_int32),
                ("max_iters", ctypes.c_int32)]


STOPS = {"space_saving": 0, "e_max": 1}


class abj_discord_info(ctypes.Structure):
    _fields_ = [("rows_exact", ctypes.c_int64), ("rounds", ctypes.c_int32), ("certified", ctypes.c_int32)]


class abj_server_opts(ctypes.Structure):
    _fields_ = [("tier", ctypes.c_int32), ("max_slots", ctypes.c_int32), ("mem_budget", ctypes.c_int64),
                ("backend", ctypes.c_int32), ("sim_n_ms", ctypes.c_int32), ("sim_ms", ctypes.c_int32 * 8),
                ("sim_dict_windows", ctypes.c_int64), ("sim_pairs_per_s", ctypes.c_double)]


class abj_req_stats(ctypes.Structure):
    _fields_ = [("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("pairs", ctypes.c_int64), ("status", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("t_device_done", ctypes.c_double)]


class abj_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("canceled", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("batches", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("busy_s", ctypes.c_double), ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("max_s", ctypes.c_double)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def header_functions():
    """Names of the functions declared in include/abjoin.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                                 src, flags=re.M)))


def lib():
    """Load libabjoin.so (raises FileNotFoundError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} is missing: build it with `python -m paper_2112_12965_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.abj_version.restype = ctypes.c_int
        L.abj_last_error.restype = ctypes.c_char_p
        L.abj_init.argtypes = [ctypes.c_int]
        L.abj_window_stats.argtypes = [_vp, _i64, _i32, _vp, _vp, _vp, _vp]
        L.ab_join.argtypes = [_vp, _i64, _vp, _i64, ctypes.POINTER(_i64), _i32, _i32, _vp, _vp,
                              ctypes.POINTER(abj_opts), _vp]
        L.ab_join_noalloc.argtypes = L.ab_join.argtypes
        L.self_join.argtypes = [_vp, _i64, _i32, _i64, _vp, _vp, _vp, ctypes.POINTER(abj_opts), _vp]
        L.dict_build.argtypes = [_vp, _i64, _i32, ctypes.POINTER(abj_learn_opts), ctypes.POINTER(_i64), _i32,
                                 ctypes.POINTER(_i32), ctypes.POINTER(_i64), _i32, ctypes.POINTER(_i32), _vp,
                                 ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double), _vp, _vp]
        L.topk_discords.argtypes = [_vp, _i64, _i32, _i64, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_float),
                                    ctypes.POINTER(_i32), _vp]
        L.discords.argtypes = [_vp, _i64, _i32, _vp, ctypes.c_double, _vp, _i64, ctypes.POINTER(_i64), _i32, _i32,
                               _i64, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_i64),
                               ctypes.POINTER(_i32), ctypes.POINTER(abj_discord_info), _vp]
        L.abj_profile_enable.argtypes = [ctypes.c_int]
        L.abj_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        L.abj_dict_create.argtypes = [_vp, _i64, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_i64),
                                      ctypes.POINTER(_i32), _i32, ctypes.POINTER(_vp)]
        L.abj_dict_source_index.argtypes = [_vp, _vp, _i64, _vp, _vp]
        L.abj_dict_free.argtypes = [_vp]
        L.ab_join_dict.argtypes = [_vp, _vp, _i64, _i32, _vp, _vp, ctypes.POINTER(abj_opts), _vp]
        L.abj_server_create.argtypes = [_vp, ctypes.POINTER(abj_server_opts), ctypes.POINTER(_vp)]
        L.abj_submit.argtypes = [_vp, _vp, _i64, _i32, ctypes.POINTER(ctypes.c_uint64)]
        L.abj_wait.argtypes = [_vp, ctypes.c_uint64, _i32]
        L.abj_submit_borrowed.argtypes = [_vp, _vp, _i64, _i32, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)]
        L.abj_result.argtypes = [_vp, ctypes.c_uint64, _vp, _vp, ctypes.POINTER(abj_req_stats)]
        L.abj_cancel.argtypes = [_vp, ctypes.c_uint64]
        L.abj_server_drain.argtypes = [_vp, _i32]
        L.abj_server_stats_get.argtypes = [_vp, ctypes.POINTER(abj_server_stats)]
        L.abj_server_destroy.argtypes = [_vp]
        for f in ("abj_init", "abj_window_stats", "ab_join", "ab_join_noalloc", "self_join", "dict_build", "topk_discords", "discords",
                  "abj_profile_enable", "abj_profile_read",
                  "abj_dict_create", "abj_dict_source_index", "abj_dict_free", "ab_join_dict", "abj_server_create", "abj_submit",
                  "abj_submit_borrowed", "abj_wait", "abj_result", "abj_cancel", "abj_server_drain",
                  "abj_server_stats_get", "abj_server_destroy"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().abj_last_error().decode(errors="replace")


def _check(rc: int):
    if rc != ABJ_OK:
        raise AbjError(rc, last_error())


def _stream_ptr(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(x, name):
    import torch

    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float64 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return x


def _bounds(seg_bounds):
    b = np.ascontiguousarray(np.asarray(seg_bounds, dtype=np.int64))
    return b, b.ctypes.data_as(ctypes.POINTER(_i64)), len(b) - 1


def ab_join(query, dictionary, seg_bounds: Sequence[int], m: int, tier: str = "fp32", refine_k: int = 0,
            out: Optional[tuple] = None, stream=None, pearson: bool = False, no_refine: bool = False):
    """Matrix profile of ``query`` against the windows of a concatenated dictionary.

    ``query``/``dictionary``: float64 CUDA tensors; ``seg_bounds``: host int64
    offsets (``[0, len(dictionary)]`` for a plain AB-join).  Returns
    ``(P, I)``: float32 distances and int64 indices (CUDA tensors), enqueued on
    the current stream.  ``pearson``: P holds the correlation of the nearest
    window instead of its distance.  ``no_refine`` (16-bit tiers): skip the
    FP64 re-check and report the distance implied by the best 16-bit score.
    """
    import torch

    q = _dev_f64(query, "query")
    d = _dev_f64(dictionary, "dictionary")
    b, bp, nseg = _bounds(seg_bounds)
    W = max(q.numel() - m + 1, 0)
    if out is None:
        P = torch.empty(W, dtype=torch.float32, device=q.device)
        I = torch.empty(W, dtype=torch.int64, device=q.device)
    else:
        P, I = out
    o = abj_opts(TIERS[tier], int(refine_k),
                 (ABJ_FLAG_PEARSON if pearson else 0) | (ABJ_FLAG_NO_REFINE if no_refine else 0), 0)
    rc = lib().ab_join(q.data_ptr(), q.numel(), d.data_ptr(), d.numel(), bp, nseg, int(m),
                       P.data_ptr() if W else None, I.data_ptr() if W else None, ctypes.byref(o),
                       _stream_ptr(stream))
    _check(rc)
    return P, I


def self_join(x, m: int, excl: int = -1, stream=None, pearson: bool = False):
    """Self-join matrix profile of ``x`` with trivial matches ``|i - j| <= excl``
    excluded (``excl < 0``: m // 2).  Returns ``(P, I, P64)`` CUDA tensors."""
    import torch

    x = _dev_f64(x, "x")
    W = max(x.numel() - m + 1, 0)
    P = torch.empty(W, dtype=torch.float32, device=x.device)
    I = torch.empty(W, dtype=torch.int64, device=x.device)
    P64 = torch.empty(W, dtype=torch.float64, device=x.device)
    o = abj_opts(0, 0, ABJ_FLAG_PEARSON if pearson else 0, 0)
    _check(lib().self_join(x.data_ptr(), x.numel(), int(m), int(excl), P.data_ptr() if W else None,
                           I.data_ptr() if W else None, P64.data_ptr() if W else None, ctypes.byref(o),
                           _stream_ptr(stream)))
    return P, I, P64


def dict_build(series, m: int, context: float = 1.5, stop: str = "space_saving", value: float = 0.9,
               max_iters: int = 0, stream=None):
    """Learning phase (Alg. 1) on the GPU.

    Returns a dict with ``segments`` (list of [start, end) ranges of the
    series), ``chosen`` (windows in the order chosen), ``dictionary`` (CUDA
    float64 tensor, the concatenated segments), ``bounds`` (its segment
    offsets), ``orig_start`` (segment starts in the series), ``e_max`` and
    ``p_b`` (the self-join profile, CUDA float64).
    """
    import torch

    x = _dev_f64(series, "series")
    n = x.numel()
    W = max(n - m + 1, 0)
    nseg, nch, nd, em = _i32(0), _i32(0), _i64(0), ctypes.c_double(0.0)
    o = abj_learn_opts(float(context), float(value), STOPS[stop], int(max_iters))
    # sizing call: upper bounds on the segments, choices and dictionary length
    _check(lib().dict_build(None, n, int(m), ctypes.byref(o), None, 0, ctypes.byref(nseg), None, 0,
                            ctypes.byref(nch), None, ctypes.byref(nd), None, None, None))
    max_seg, max_ch = max(nseg.value, 1), max(nch.value, 1)
    segs = np.zeros(2 * max_seg, dtype=np.int64)
    chosen = np.zeros(max_ch, dtype=np.int64)
    d = torch.empty(max(nd.value, 1), dtype=torch.float64, device=x.device)
    pb = torch.empty(max(W, 1), dtype=torch.float64, device=x.device)
    _check(lib().dict_build(x.data_ptr(), n, int(m), ctypes.byref(o), segs.ctypes.data_as(ctypes.POINTER(_i64)),
                            max_seg, ctypes.byref(nseg), chosen.ctypes.data_as(ctypes.POINTER(_i64)),
                            max_ch, ctypes.byref(nch), d.data_ptr(), ctypes.byref(nd), ctypes.byref(em),
                            pb.data_ptr() if W else None, _stream_ptr(stream)))
    sg = [(int(segs[2 * k]), int(segs[2 * k + 1])) for k in range(nseg.value)]
    bounds = np.concatenate([[0], np.cumsum([b - a for a, b in sg])]).astype(np.int64)
    return dict(segments=sg, chosen=chosen[:nch.value].copy(), dictionary=d[:nd.value], bounds=bounds,
                orig_start=np.array([a for a, _ in sg], dtype=np.int64), e_max=em.value, p_b=pb[:W])


def _dev_f32(x, name):
    import torch

    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return x


def topk_discords(P, K: int, excl: int, stream=None):
    """Greedy top-K discords of a profile (float32 CUDA tensor): (rows, values)."""
    P = _dev_f32(P, "P")
    rows = np.zeros(K, dtype=np.int64)
    vals = np.zeros(K, dtype=np.float32)
    n = _i32(0)
    _check(lib().topk_discords(P.data_ptr(), P.numel(), int(K), int(excl), rows.ctypes.data_as(ctypes.POINTER(_i64)),
                               vals.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(n),
                               _stream_ptr(stream)))
    return rows[:n.value].copy(), vals[:n.value].copy()


def discords(query, P_hat, e_max: float, ref, ref_bounds, m: int, K: int, excl: int = -1, stream=None):
    """Exact top-K discords of ``query`` against ``ref`` from the dictionary join ``P_hat``.

    Returns a dict with ``rows``, ``values`` (exact distances), ``neighbors``
    (nearest windows in ``ref``), ``rows_exact``, ``rounds`` and ``certified``.
    """
    q = _dev_f64(query, "query")
    r = _dev_f64(ref, "ref")
    Ph = _dev_f32(P_hat, "P_hat")
    b, bp, nseg = _bounds(ref_bounds)
    rows = np.zeros(K, dtype=np.int64)
    vals = np.zeros(K, dtype=np.float32)
    nn = np.zeros(K, dtype=np.int64)
    n = _i32(0)
    info = abj_discord_info()
    _check(lib().discords(q.data_ptr(), q.numel(), int(m), Ph.data_ptr(), float(e_max), r.data_ptr(), r.numel(), bp,
                          nseg, int(K), int(excl), rows.ctypes.data_as(ctypes.POINTER(_i64)),
                          vals.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                          nn.ctypes.data_as(ctypes.POINTER(_i64)), ctypes.byref(n), ctypes.byref(info),
                          _stream_ptr(stream)))
    k = n.value
    return dict(rows=rows[:k].copy(), values=vals[:k].copy(), neighbors=nn[:k].copy(), rows_exact=info.rows_exact,
                rounds=info.rounds, certified=info.certified)


def window_stats(x, m: int, stream=None):
    """(mean, population deviation, flags) of every length-m window of ``x``."""
    import torch

    x = _dev_f64(x, "x")
    W = max(x.numel() - m + 1, 0)
    mu = torch.empty(W, dtype=torch.float64, device=x.device)
    sig = torch.empty(W, dtype=torch.float64, device=x.device)
    fl = torch.empty(W, dtype=torch.uint8, device=x.device)
    _check(lib().abj_window_stats(x.data_ptr(), x.numel(), int(m), mu.data_ptr() if W else None,
                                  sig.data_ptr() if W else None, fl.data_ptr() if W else None,
                                  _stream_ptr(stream)))
    return mu, sig, fl


class Dictionary:
    """A dictionary kept resident in device memory (library-owned), with window
    statistics precomputed for every window length in ``ms``."""

    def __init__(self, dictionary, seg_bounds, ms, orig_start=None):
        import torch

        if isinstance(dictionary, torch.Tensor):
            x = dictionary.detach().to(torch.float64).contiguous()
            ptr, n, self._keep = x.data_ptr(), x.numel(), x
        else:
            x = np.ascontiguousarray(np.asarray(dictionary, dtype=np.float64))
            ptr, n, self._keep = x.ctypes.data, len(x), x
        b, bp, nseg = _bounds(seg_bounds)
        m_arr = (ctypes.c_int32 * len(ms))(*[int(v) for v in ms])
        op = None
        if orig_start is not None:
            self._orig = np.ascontiguousarray(np.asarray(orig_start, dtype=np.int64))
            if len(self._orig) != nseg:
                raise ValueError("orig_start needs one entry per segment")
            op = self._orig.ctypes.data_as(ctypes.POINTER(_i64))
        h = ctypes.c_void_p()
        _check(lib().abj_dict_create(ptr, n, bp, nseg, op, m_arr, len(ms), ctypes.byref(h)))
        self.handle = h
        self.ms = tuple(int(v) for v in ms)
        self.n = n
        self.bounds = b

    def join(self, query, m, tier="fp32", refine_k=0, no_refine=False, out=None, stream=None, pearson=False):
        import torch

        q = _dev_f64(query, "query")
        W = max(q.numel() - m + 1, 0)
        if out is None:
            P = torch.empty(W, dtype=torch.float32, device=q.device)
            I = torch.empty(W, dtype=torch.int64, device=q.device)
        else:
            P, I = out
        o = abj_opts(TIERS[tier], int(refine_k),
                     (ABJ_FLAG_NO_REFINE if no_refine else 0) | (ABJ_FLAG_PEARSON if pearson else 0), 0)
        _check(lib().ab_join_dict(self.handle, q.data_ptr(), q.numel(), int(m), P.data_ptr() if W else None,
                                  I.data_ptr() if W else None, ctypes.byref(o), _stream_ptr(stream)))
        return P, I

    def source_index(self, I, out=None, stream=None):
        """Positions in the source series of dictionary indices ``I`` (int64
        CUDA tensor; -1 stays -1)."""
        import torch

        if not isinstance(I, torch.Tensor) or not I.is_cuda or I.dtype != torch.int64 or not I.is_contiguous():
            raise TypeError("I must be a contiguous int64 CUDA tensor")
        if out is None:
            out = torch.empty_like(I)
        _check(lib().abj_dict_source_index(self.handle, I.data_ptr() if I.numel() else None, I.numel(),
                                           out.data_ptr() if I.numel() else None, _stream_ptr(stream)))
        return out

    def close(self):
        if self.handle:
            lib().abj_dict_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching join server over a resident Dictionary.

    ``backend="sim"`` runs the scheduler without any GPU call (for tests):
    then ``dictionary`` is None and ``sim_ms`` / ``sim_dict_windows`` /
    ``sim_pairs_per_s`` describe the simulated dictionary and speed.
    """

    def __init__(self, dictionary=None, tier="fp32", max_slots=64, mem_budget=8 << 30, backend="gpu",
                 sim_ms=(64, 128, 256), sim_dict_windows=60000, sim_pairs_per_s=1e12):
        o = abj_server_opts()
        o.tier = TIERS[tier]
        o.max_slots = int(max_slots)
        o.mem_budget = int(mem_budget)
        o.backend = {"gpu": 0, "sim": 1}[backend]
        o.sim_n_ms = len(sim_ms)
        for k, v in enumerate(sim_ms):
            o.sim_ms[k] = int(v)
        o.sim_dict_windows = int(sim_dict_windows)
        o.sim_pairs_per_s = float(sim_pairs_per_s)
        h = ctypes.c_void_p()
        _check(lib().abj_server_create(dictionary.handle if dictionary is not None else None, ctypes.byref(o),
                                       ctypes.byref(h)))
        self.handle = h
        self._dict = dictionary
        self._reqs = {}  # id -> (rows, borrowed buffers or None)

    def submit(self, query, m, copy=False):
        """Queue a join of `query` (host array) at window length m; returns the id.

        By default the request borrows the query and result buffers (the
        server reads and writes them on its own thread; this object keeps
        them alive until result()); copy=True has the server copy the query
        at submission instead.
        """
        q = np.ascontiguousarray(np.asarray(query, dtype=np.float64))
        W = len(q) - int(m) + 1
        rid = ctypes.c_uint64()
        if copy:
            _check(lib().abj_submit(self.handle, q.ctypes.data, len(q), int(m), ctypes.byref(rid)))
            self._reqs[rid.value] = (W, None)
        else:
            P = np.empty(max(W, 1), dtype=np.float32)
            I = np.empty(max(W, 1), dtype=np.int64)
            _check(lib().abj_submit_borrowed(self.handle, q.ctypes.data, len(q), int(m), P.ctypes.data,
                                             I.ctypes.data, ctypes.byref(rid)))
            self._reqs[rid.value] = (W, (q, P, I))
        return rid.value

    def wait(self, rid, timeout_ms=-1):
        """Status code: ABJ_OK, ABJ_ECANCELED, ABJ_ETIMEOUT, ..."""
        return lib().abj_wait(self.handle, ctypes.c_uint64(rid), int(timeout_ms))

    def result(self, rid):
        """(P, I, stats) of a finished request (numpy arrays, dict)."""
        W, keep = self._reqs[rid]
        if keep is None:
            P = np.empty(W, dtype=np.float32)
            I = np.empty(W, dtype=np.int64)
            ptrs = (P.ctypes.data, I.ctypes.data)
        else:
            P, I = keep[1][:W], keep[2][:W]
            ptrs = (None, None)
        st = abj_req_stats()
        rc = lib().abj_result(self.handle, ctypes.c_uint64(rid), ptrs[0], ptrs[1], ctypes.byref(st))
        stats = {f: getattr(st, f) for f, _ in abj_req_stats._fields_}
        if rc not in (ABJ_EBUSY, ABJ_ENOTFOUND):
            del self._reqs[rid]  # the server has forgotten the request
        if rc != ABJ_OK:
            raise AbjError(rc, last_error())
        return P, I, stats

    def cancel(self, rid):
        return lib().abj_cancel(self.handle, ctypes.c_uint64(rid))

    def drain(self, timeout_ms=-1):
        return lib().abj_server_drain(self.handle, int(timeout_ms))

    def stats(self):
        st = abj_server_stats()
        _check(lib().abj_server_stats_get(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in abj_server_stats._fields_}

    def close(self):
        if self.handle:
            lib().abj_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
