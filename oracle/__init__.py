"""CPU oracle for top-k weighted triangles — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The GPU library never links, loads or calls it, and the two share no
code.  Everything here follows the problem statement of Sec. 1 (Eq. 1 and the special means
named after it) and weighted edge sampling (Alg. 3, Prop. 1); see ``oracle.c`` for the
readings taken where the paper is silent (tie order, fewer than k triangles, the sampling
exponent for p <= 0).

The numeric heavy lifting is plain C (``oracle.c``) compiled with gcc into
``liboracle.so``; this file only marshals arguments.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# status codes (same meaning as the library's, defined independently)
OK, E_ARG, E_SELF_LOOP, E_DUP_EDGE, E_ZERO_WEIGHT, E_VERTEX_RANGE, E_NOMEM = 0, -1, -2, -3, -4, -5, -6
FILTER_NONE, FILTER_EDGE_MARK, FILTER_VERTEX_MARK = 0, 1, 2
EXACT_P = (-math.inf, 0.0, 1.0, 2.0, math.inf)


def build(force: bool = True) -> str:
    """Compile liboracle.so (gcc, -O2, OpenMP, strict IEEE: no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, u32, dbl, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_int
        p32 = ctypes.POINTER(ctypes.c_uint32)
        p64 = ctypes.POINTER(ctypes.c_uint64)
        pd = ctypes.POINTER(ctypes.c_double)
        p8 = ctypes.POINTER(ctypes.c_uint8)
        lib.orc_mode.argtypes = [dbl]
        lib.orc_mode.restype = i32
        lib.orc_score.argtypes = [dbl, u32, u32, u32, p64, p64]
        lib.orc_score.restype = dbl
        lib.orc_validate.argtypes = [u64, u64, p32, p32, p32]
        lib.orc_validate.restype = i32
        lib.orc_topk.argtypes = [u64, u64, p32, p32, p32, u64, dbl, i32, i32, p8, p32, p32, p32, pd, p64, p64,
                                 p64, p64]
        lib.orc_topk.restype = i32
        lib.orc_list.argtypes = [u64, u64, p32, p32, p32, u64, p32, p32, p32, p32, p64]
        lib.orc_list.restype = i32
        lib.orc_topk_marked.argtypes = [u64, u64, p32, p32, p32, u64, dbl, i32, p8, p8, p32, p32, p32, pd, p64,
                                        p64, p64, p64]
        lib.orc_topk_marked.restype = i32
        lib.orc_topk_on_marked_edges.argtypes = lib.orc_topk_marked.argtypes
        lib.orc_topk_on_marked_edges.restype = i32
        lib.orc_cliques.argtypes = [u64, u64, p32, p32, p32, i32, u64, dbl, i32, p8, p32, pd, p64, p64]
        lib.orc_cliques.restype = i32
        lib.orc_es_draw.argtypes = [u64, p32, dbl, u64, u64, p8, p64]
        lib.orc_es_draw.restype = i32
        lib.orc_es_draw_q.argtypes = [u64, p32, dbl, u64, u64, p8, p64]
        lib.orc_es_draw_q.restype = i32
        lib.orc_es_prefix_f64.argtypes = [u64, p32, dbl, pd]
        lib.orc_es_prefix_f64.restype = i32
        lib.orc_sample_exponent.argtypes = [dbl]
        lib.orc_sample_exponent.restype = dbl
        lib.orc_splitmix64_at.argtypes = [u64, u64]
        lib.orc_splitmix64_at.restype = u64
        _lib = lib
    return _lib


def _arr(a, dtype):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    return a


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _edges(src, dst, w):
    s, d, ww = _arr(src, np.uint32), _arr(dst, np.uint32), _arr(w, np.uint32)
    if not (s.shape == d.shape == ww.shape) or s.ndim != 1:
        raise ValueError("src, dst, w must be 1-D arrays of equal length")
    return s, d, ww


def score(p: float, a: int, b: int, c: int):
    """(exact order key as a Python int, FP64 score) of a triangle with weights a, b, c."""
    hi, lo = ctypes.c_uint64(0), ctypes.c_uint64(0)
    s = _load().orc_score(float(p), a, b, c, ctypes.byref(hi), ctypes.byref(lo))
    return (hi.value << 64) | lo.value, s


def validate(n, src, dst, w) -> int:
    s, d, ww = _edges(src, dst, w)
    return _load().orc_validate(n, s.shape[0], _ptr(s, ctypes.c_uint32), _ptr(d, ctypes.c_uint32),
                                _ptr(ww, ctypes.c_uint32))


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def topk(n, src, dst, w, k: int, p: float, nthreads: int = 0, edge_mark=None, vertex_mark=None,
         from_marked_edges: bool = False):
    """Top-k triangles.  Returns dict(i, j, l, score, key, n_out, total).  With edge_mark (per
    input edge) only triangles with a marked edge are admitted, with vertex_mark (per vertex)
    only triangles with a marked vertex; with both, triangles that satisfy both.
    from_marked_edges: the same result, the triangles found from the marked edges (no full
    enumeration; edge_mark required)."""
    s, d, ww = _edges(src, dst, w)
    m = s.shape[0]
    em = vm = None
    if edge_mark is not None:
        em = _arr(edge_mark, np.uint8)
        assert em.shape[0] == m
    if vertex_mark is not None:
        vm = _arr(vertex_mark, np.uint8)
        assert vm.shape[0] == n
    kk = max(int(k), 0)
    oi, oj, ol = (np.zeros(max(kk, 1), np.uint32) for _ in range(3))
    osc = np.zeros(max(kk, 1), np.float64)
    khi, klo = np.zeros(max(kk, 1), np.uint64), np.zeros(max(kk, 1), np.uint64)
    nout, tot = ctypes.c_uint64(0), ctypes.c_uint64(0)
    fn = _load().orc_topk_on_marked_edges if from_marked_edges else _load().orc_topk_marked
    if from_marked_edges and em is None:
        raise ValueError("from_marked_edges needs edge_mark")
    rc = fn(n, m, _ptr(s, ctypes.c_uint32), _ptr(d, ctypes.c_uint32),
                                 _ptr(ww, ctypes.c_uint32), kk, float(p), int(nthreads),
                                 None if em is None else _ptr(em, ctypes.c_uint8),
                                 None if vm is None else _ptr(vm, ctypes.c_uint8),
                                 _ptr(oi, ctypes.c_uint32), _ptr(oj, ctypes.c_uint32), _ptr(ol, ctypes.c_uint32),
                                 _ptr(osc, ctypes.c_double), _ptr(khi, ctypes.c_uint64),
                                 _ptr(klo, ctypes.c_uint64), ctypes.byref(nout), ctypes.byref(tot))
    if rc != OK:
        raise OracleError(rc)
    r = int(nout.value)
    keys = [(int(h) << 64) | int(lo) for h, lo in zip(khi[:r], klo[:r])]
    return {"i": oi[:r].copy(), "j": oj[:r].copy(), "l": ol[:r].copy(), "score": osc[:r].copy(), "key": keys,
            "n_out": r, "total": int(tot.value)}


def list_triangles(n, src, dst, w, cap: int | None = None):
    """All triangles (i<j<l, unordered) with weights (w_ij, w_il, w_jl).  Small graphs only."""
    s, d, ww = _edges(src, dst, w)
    lib = _load()
    cnt = ctypes.c_uint64(0)
    if cap is None:
        rc = lib.orc_list(n, s.shape[0], _ptr(s, ctypes.c_uint32), _ptr(d, ctypes.c_uint32),
                          _ptr(ww, ctypes.c_uint32), 0, None, None, None, None, ctypes.byref(cnt))
        if rc != OK:
            raise OracleError(rc)
        cap = int(cnt.value)
    oi, oj, ol = (np.zeros(max(cap, 1), np.uint32) for _ in range(3))
    ow = np.zeros(3 * max(cap, 1), np.uint32)
    rc = lib.orc_list(n, s.shape[0], _ptr(s, ctypes.c_uint32), _ptr(d, ctypes.c_uint32), _ptr(ww, ctypes.c_uint32),
                      cap, _ptr(oi, ctypes.c_uint32), _ptr(oj, ctypes.c_uint32), _ptr(ol, ctypes.c_uint32),
                      _ptr(ow, ctypes.c_uint32), ctypes.byref(cnt))
    if rc != OK:
        raise OracleError(rc)
    t = min(int(cnt.value), cap)
    return oi[:t].copy(), oj[:t].copy(), ol[:t].copy(), ow[:3 * t].reshape(t, 3).copy()


def count_triangles(n, src, dst, w) -> int:
    return topk(n, src, dst, w, 0, 1.0)["total"]


def sample_exponent(p: float) -> float:
    return _load().orc_sample_exponent(float(p))


def splitmix64(seed: int, i: int) -> int:
    return int(_load().orc_splitmix64_at(seed & (2**64 - 1), i))


def es_draw(w, p: float, budget: int, seed: int, return_draws: bool = False, q: float | None = None):
    """Alg. 3's edge draws with the sampling exponent of p, or with q when it is given.
    Returns the per-edge mark array (and the draw sequence)."""
    ww = _arr(w, np.uint32)
    m = ww.shape[0]
    mark = np.zeros(max(m, 1), np.uint8)
    draws = np.zeros(max(budget, 1), np.uint64) if return_draws else None
    args = (m, _ptr(ww, ctypes.c_uint32))
    rest = (int(budget), seed & (2**64 - 1), _ptr(mark, ctypes.c_uint8),
            None if draws is None else _ptr(draws, ctypes.c_uint64))
    if q is None:
        rc = _load().orc_es_draw(*args, float(p), *rest)
    else:
        rc = _load().orc_es_draw_q(*args, float(q), *rest)
    if rc != OK:
        raise OracleError(rc)
    mark = mark[:m]
    return (mark, draws[:budget]) if return_draws else mark


def es_prefix_f64(w, q: float) -> np.ndarray:
    """The FP64 prefix sums of w^q that the draws of a non-integer q search."""
    ww = _arr(w, np.uint32)
    P = np.zeros(max(ww.shape[0], 1), np.float64)
    rc = _load().orc_es_prefix_f64(ww.shape[0], _ptr(ww, ctypes.c_uint32), float(q), _ptr(P, ctypes.c_double))
    if rc != OK:
        raise OracleError(rc)
    return P[: ww.shape[0]]


def sample_heavy_triangles(n, src, dst, w, k: int, p: float, budget: int, seed: int, nthreads: int = 0,
                           q: float | None = None):
    """Alg. 3 end to end: draws, union of the triangles on the drawn edges, top-k by m_p."""
    mark = es_draw(w, p, budget, seed, q=q)
    out = topk(n, src, dst, w, k, p, nthreads=nthreads, edge_mark=mark)
    out["distinct_edges"] = int(mark.sum())
    return out


def cliques(n, src, dst, w, size: int, k: int, p: float, edge_mark=None, nthreads: int = 0):
    """Top-k cliques of `size` (4 or 5) vertices by the p-mean of their edge weights (Sec. 4.5),
    optionally only those holding a marked edge.  Returns dict(v: [n_out, size], score, n_out,
    total)."""
    s, d, ww = _edges(src, dst, w)
    em = None if edge_mark is None else _arr(edge_mark, np.uint8)
    kk = max(int(k), 0)
    ov = np.zeros(5 * max(kk, 1), np.uint32)
    osc = np.zeros(max(kk, 1), np.float64)
    nout, tot = ctypes.c_uint64(0), ctypes.c_uint64(0)
    rc = _load().orc_cliques(n, s.shape[0], _ptr(s, ctypes.c_uint32), _ptr(d, ctypes.c_uint32),
                             _ptr(ww, ctypes.c_uint32), int(size), kk, float(p), int(nthreads),
                             None if em is None else _ptr(em, ctypes.c_uint8), _ptr(ov, ctypes.c_uint32),
                             _ptr(osc, ctypes.c_double), ctypes.byref(nout), ctypes.byref(tot))
    if rc != OK:
        raise OracleError(rc)
    r = int(nout.value)
    return {"v": ov[: 5 * r].reshape(r, 5)[:, :size].copy(), "score": osc[:r].copy(), "n_out": r,
            "total": int(tot.value)}


def sample_heavy_cliques(n, src, dst, w, size: int, k: int, p: float, budget: int, seed: int, q=None,
                         nthreads: int = 0):
    """Edge sampling extended to cliques (Sec. 4.5): the draws of Alg. 3, then the top-k cliques
    holding a drawn edge."""
    mark = es_draw(w, p, budget, seed, q=q)
    return cliques(n, src, dst, w, size, k, p, edge_mark=mark, nthreads=nthreads)
