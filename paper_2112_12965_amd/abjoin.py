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
        for f in ("abj_init", "abj_window_stats", "ab_join"):
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
            out: Optional[tuple] = None, stream=None):
    """Matrix profile of ``query`` against the windows of a concatenated dictionary.

    ``query``/``dictionary``: float64 CUDA tensors; ``seg_bounds``: host int64
    offsets (``[0, len(dictionary)]`` for a plain AB-join).  Returns
    ``(P, I)``: float32 distances and int64 indices (CUDA tensors), enqueued on
    the current stream.
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
    o = abj_opts(TIERS[tier], int(refine_k), 0, 0)
    rc = lib().ab_join(q.data_ptr(), q.numel(), d.data_ptr(), d.numel(), bp, nseg, int(m),
                       P.data_ptr() if W else None, I.data_ptr() if W else None, ctypes.byref(o),
                       _stream_ptr(stream))
    _check(rc)
    return P, I


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
