"""The paper's exact method on the CPU (libtopktri_dhl.so, include/topktri_dhl.h): the dynamic
heavy-light algorithm (Alg. 2) and Auto-HL (Sec. 3.3).  ctypes marshalling only."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import Triangle, TopKError, _result, _u32
from ._build import DHL_LIB

_lib = None


class DHLStats(ctypes.Structure):
    _fields_ = [("enumerated", ctypes.c_uint64), ("h_moves", ctypes.c_uint64), ("l_moves", ctypes.c_uint64),
                ("lookups", ctypes.c_uint64), ("final_h", ctypes.c_uint64), ("final_l", ctypes.c_uint64),
                ("sort_ms", ctypes.c_double), ("build_ms", ctypes.c_double), ("loop_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def library():
    global _lib
    if _lib is None:
        if not os.path.exists(DHL_LIB):
            raise FileNotFoundError(f"{DHL_LIB} is not built (run __graft_entry__.build())")
        lib = ctypes.CDLL(DHL_LIB)
        p32 = ctypes.POINTER(ctypes.c_uint32)
        lib.dhl_topk_triangles.argtypes = [ctypes.c_uint32, ctypes.c_uint64, p32, p32, p32, ctypes.c_uint32,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Triangle),
                                           p32, ctypes.POINTER(DHLStats)]
        lib.dhl_topk_triangles.restype = ctypes.c_int
        lib.dhl_last_error.argtypes = []
        lib.dhl_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def topk(n, src, dst, w, k: int, p: float, alpha: float = 1.25, threads: int = 0):
    """Exact top-k triangles by m_p with Alg. 2 (alpha > 0) or Auto-HL (alpha = 0).
    Returns dict(i, j, l, score, n_out, stats)."""
    lib = library()
    s, d, ww = _u32(src), _u32(dst), _u32(w)
    if not (s.shape == d.shape == ww.shape) or s.ndim != 1:
        raise ValueError("src, dst, w must be 1-D arrays of equal length")
    p32 = ctypes.POINTER(ctypes.c_uint32)
    buf = (Triangle * max(int(k), 1))()
    n_out = ctypes.c_uint32(0)
    st = DHLStats()
    rc = lib.dhl_topk_triangles(int(n), int(s.shape[0]), s.ctypes.data_as(p32), d.ctypes.data_as(p32),
                                ww.ctypes.data_as(p32), int(k), float(p), float(alpha), int(threads), buf,
                                ctypes.byref(n_out), ctypes.byref(st))
    if rc != 0:
        raise TopKError(rc, lib.dhl_last_error().decode(errors="replace"))
    out = _result(buf, n_out.value)
    out["stats"] = st.as_dict()
    return out
