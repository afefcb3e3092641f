"""Top-k weighted triangles on AMD MI355X: a thin ctypes binding over libtopktri.so.

Every step of the computation runs in the HIP library (``csrc/``); this module only marshals
arguments.  The C ABI is declared in ``include/topktri.h``.  Inputs may be NumPy arrays (host)
or torch CUDA tensors (device, loaded on the tensor's current stream).

If the library has not been built, importing works but any call raises ``LibraryMissing``:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from ._build import LIB as LIB_PATH, build  # noqa: F401

_lib = None

TT_OK, TT_E_ARG, TT_E_SELF_LOOP, TT_E_DUP_EDGE, TT_E_ZERO_WEIGHT = 0, -1, -2, -3, -4
TT_E_VERTEX_RANGE, TT_E_NOMEM, TT_E_DEVICE, TT_E_BUDGET, TT_E_TOO_LARGE = -5, -6, -7, -8, -9

EXPORTED = ("graph_load", "graph_load_device", "topk_triangles", "topk_triangles_ex", "sample_heavy_triangles",
            "sample_heavy_triangles_ex", "graph_num_vertices", "graph_num_edges", "graph_device_bytes",
            "graph_free", "tt_last_error", "server_create", "server_request_bytes", "server_submit", "server_poll",
            "server_wait", "server_info", "server_destroy", "batch_load", "batch_load_device", "batch_topk",
            "batch_topk_ex", "batch_num_configs", "batch_num_graphs", "batch_free", "tt_trim_cache",
            "topk_triangles_noalloc", "shl_topk_triangles", "sample_triangles_by", "sample_heavy_cliques", "server_scratch_bytes")
TT_SAMPLE_WEDGE, TT_SAMPLE_PATH = 1, 2
TT_BATCH_EAGER = 1


class Triangle(ctypes.Structure):
    _fields_ = [("i", ctypes.c_uint32), ("j", ctypes.c_uint32), ("l", ctypes.c_uint32), ("_pad", ctypes.c_uint32),
                ("score", ctypes.c_double)]


class Clique(ctypes.Structure):
    _fields_ = [("v", ctypes.c_uint32 * 5), ("size", ctypes.c_uint32), ("score", ctypes.c_double)]


class QueryStats(ctypes.Structure):
    _fields_ = [("candidate_edges", ctypes.c_uint64), ("intersected_entries", ctypes.c_uint64),
                ("triangles_emitted", ctypes.c_uint64), ("edges_streamed", ctypes.c_uint64),
                ("distinct_sampled", ctypes.c_uint64), ("passes", ctypes.c_uint32), ("restarts", ctypes.c_uint32),
                ("enum_ms", ctypes.c_double), ("select_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("enum_kernel_ms", ctypes.c_double), ("sample_ms", ctypes.c_double),
                ("bound_order", ctypes.c_uint64), ("heavy_candidates", ctypes.c_uint64),
                ("heavy_overflow", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchStats(ctypes.Structure):
    _fields_ = [("candidate_edges", ctypes.c_uint64), ("intersected_entries", ctypes.c_uint64),
                ("triangles_emitted", ctypes.c_uint64), ("edges_streamed", ctypes.c_uint64),
                ("config", ctypes.c_uint32), ("growth", ctypes.c_uint32), ("filter_blocks", ctypes.c_uint32),
                ("intersect_blocks", ctypes.c_uint32), ("passes", ctypes.c_uint32),
                ("restart_rounds", ctypes.c_uint32), ("restarts", ctypes.c_uint32), ("merge_max", ctypes.c_uint32),
                ("launch_ms", ctypes.c_double), ("tune_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


TRI_DTYPE = np.dtype([("i", np.uint32), ("j", np.uint32), ("l", np.uint32), ("_pad", np.uint32),
                      ("score", np.float64)])
assert TRI_DTYPE.itemsize == ctypes.sizeof(Triangle) == 24


class LibraryMissing(RuntimeError):
    pass


class TopKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"status {code}: {msg}")
        self.code = code


def library():
    """Loads libtopktri.so (raises LibraryMissing if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        # torch ships its own HIP runtime with the same SONAME (libamdhip64.so.7); loading it
        # first makes the library bind to that one, so torch streams and pointers are shared
        # with a single runtime instead of two runtimes competing for the device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        u32, u64, dbl, vp, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        p32 = ctypes.POINTER(ctypes.c_uint32)
        pg = ctypes.POINTER(ctypes.c_void_p)
        ptri = ctypes.POINTER(Triangle)
        pst = ctypes.POINTER(QueryStats)
        lib.graph_load.argtypes = [u32, u64, p32, p32, p32, pg]
        lib.graph_load_device.argtypes = [u32, u64, vp, vp, vp, vp, pg]
        lib.topk_triangles.argtypes = [vp, u32, dbl, ptri, p32]
        lib.topk_triangles_ex.argtypes = [vp, u32, dbl, p32, u32, ptri, p32, pst]
        lib.topk_triangles_noalloc.argtypes = [vp, u32, dbl, ptri, p32]
        lib.shl_topk_triangles.argtypes = [vp, u32, dbl, u32, ptri, p32, ctypes.POINTER(ctypes.c_uint64)]
        lib.sample_triangles_by.argtypes = [vp, i32, u32, dbl, u64, u64, dbl, p32, ptri, p32,
                                            ctypes.POINTER(ctypes.c_uint64 * 2)]
        lib.sample_heavy_cliques.argtypes = [vp, u32, u32, dbl, u64, u64, dbl, u32, ctypes.POINTER(Clique), p32,
                                             ctypes.POINTER(ctypes.c_uint64)]
        lib.sample_heavy_triangles.argtypes = [vp, u32, dbl, u64, u64, ptri, p32]
        lib.sample_heavy_triangles_ex.argtypes = [vp, u32, dbl, u64, u64, dbl, p32, ptri, p32, pst]
        lib.graph_num_vertices.argtypes = [vp]
        lib.graph_num_vertices.restype = u32
        lib.graph_num_edges.argtypes = [vp]
        lib.graph_num_edges.restype = u64
        lib.graph_device_bytes.argtypes = [vp]
        lib.graph_device_bytes.restype = u64
        lib.graph_free.argtypes = [vp]
        lib.graph_free.restype = None
        lib.tt_last_error.argtypes = []
        lib.tt_last_error.restype = ctypes.c_char_p
        lib.tt_trim_cache.argtypes = []
        lib.tt_trim_cache.restype = u64
        p64 = ctypes.POINTER(ctypes.c_uint64)
        pint = ctypes.POINTER(ctypes.c_int)
        lib.server_create.argtypes = [vp, u32, u64, pg]
        lib.server_request_bytes.argtypes = [vp, u32, u32]
        lib.server_request_bytes.restype = u64
        lib.server_scratch_bytes.argtypes = [vp]
        lib.server_scratch_bytes.restype = u64
        lib.server_submit.argtypes = [vp, u32, dbl, p32, u32, p64]
        lib.server_poll.argtypes = [vp, u64, pint]
        lib.server_wait.argtypes = [vp, u64, ptri, p32, pst]
        lib.server_info.argtypes = [vp, p64, p64, p64, p32, p32]
        lib.server_destroy.argtypes = [vp]
        lib.server_destroy.restype = None
        pbst = ctypes.POINTER(BatchStats)
        lib.batch_load.argtypes = [u32, p32, p64, p32, p32, p32, pg]
        lib.batch_load_device.argtypes = [u32, p32, p64, vp, vp, vp, vp, pg]
        lib.batch_topk.argtypes = [vp, u32, dbl, ptri, p32]
        lib.batch_topk_ex.argtypes = [vp, u32, dbl, i32, u32, ptri, p32, pbst]
        lib.batch_num_configs.argtypes = []
        lib.batch_num_configs.restype = u32
        lib.batch_num_graphs.argtypes = [vp]
        lib.batch_num_graphs.restype = u32
        lib.batch_free.argtypes = [vp]
        lib.batch_free.restype = None
        for name in ("graph_load", "graph_load_device", "topk_triangles", "topk_triangles_ex", "topk_triangles_noalloc",
                     "shl_topk_triangles", "sample_triangles_by", "sample_heavy_cliques",
                     "sample_heavy_triangles", "sample_heavy_triangles_ex", "server_create", "server_submit",
                     "server_poll", "server_wait", "server_info", "batch_load", "batch_load_device", "batch_topk",
                     "batch_topk_ex"):
            getattr(lib, name).restype = i32
        _lib = lib
    return _lib


def _check(rc):
    if rc != TT_OK:
        raise TopKError(rc, library().tt_last_error().decode(errors="replace"))


def _u32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


def _result(buf, n):
    r = np.frombuffer(buf, dtype=TRI_DTYPE, count=n).copy() if n else np.zeros(0, TRI_DTYPE)
    return {"i": r["i"], "j": r["j"], "l": r["l"], "score": r["score"], "n_out": int(n)}


class Graph:
    """A graph resident on the GPU (the degree-oriented CSR built by graph_load)."""

    def __init__(self, n: int, src, dst, w, stream=None):
        lib = library()
        self._h = ctypes.c_void_p()
        if hasattr(src, "is_cuda") and src.is_cuda:
            import torch
            s = src.contiguous().to(torch.int32) if src.dtype != torch.int32 else src.contiguous()
            d = dst.contiguous().to(torch.int32) if dst.dtype != torch.int32 else dst.contiguous()
            ww = w.contiguous().to(torch.int32) if w.dtype != torch.int32 else w.contiguous()
            if stream is None:
                stream = torch.cuda.current_stream(src.device)
            st = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
            _check(lib.graph_load_device(int(n), int(s.numel()), ctypes.c_void_p(s.data_ptr()),
                                         ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(ww.data_ptr()), st,
                                         ctypes.byref(self._h)))
            self._keep = (s, d, ww)
        else:
            s, d, ww = _u32(src), _u32(dst), _u32(w)
            if not (s.shape == d.shape == ww.shape) or s.ndim != 1:
                raise ValueError("src, dst, w must be 1-D arrays of equal length")
            p32 = ctypes.POINTER(ctypes.c_uint32)
            _check(lib.graph_load(int(n), int(s.shape[0]), s.ctypes.data_as(p32), d.ctypes.data_as(p32),
                                  ww.ctypes.data_as(p32), ctypes.byref(self._h)))
        self.n = int(n)
        self.m = int(lib.graph_num_edges(self._h))

    @property
    def handle(self):
        return self._h

    @property
    def device_bytes(self) -> int:
        return int(library().graph_device_bytes(self._h))

    def topk(self, k: int, p: float, subset=None, with_stats: bool = False):
        """Exact top-k triangles by m_p.  Returns dict(i, j, l, score, n_out[, stats])."""
        lib = library()
        buf = (Triangle * max(int(k), 1))()
        n_out = ctypes.c_uint32(0)
        st = QueryStats()
        sub_p, sub_n = None, 0
        if subset is not None and len(subset):
            sub = _u32(subset)
            sub_p, sub_n = sub.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), int(sub.shape[0])
        _check(lib.topk_triangles_ex(self._h, int(k), float(p), sub_p, sub_n, buf, ctypes.byref(n_out),
                                     ctypes.byref(st)))
        out = _result(buf, n_out.value)
        if with_stats:
            out["stats"] = st.as_dict()
        return out

    def shl(self, k: int, p: float, tau: int):
        """Static heavy-light (Alg. 1): top-k of the triangles whose three edges weigh > tau."""
        buf = (Triangle * max(int(k), 1))()
        n_out = ctypes.c_uint32(0)
        mh = ctypes.c_uint64(0)
        _check(library().shl_topk_triangles(self._h, int(k), float(p), int(tau), buf, ctypes.byref(n_out),
                                            ctypes.byref(mh)))
        out = _result(buf, n_out.value)
        out["heavy_edges"] = int(mh.value)
        return out

    def sample_by(self, scheme: str, k: int, p: float, budget: int, seed: int, q: float | None = None,
                  return_draws: bool = False):
        """Wedge (Alg. 4) or path (Alg. 5) sampling: top-k of the distinct triangles the draws
        close.  scheme: "wedge" or "path".  return_draws adds "draws" (budget x 4 uint32)."""
        sc = {"wedge": TT_SAMPLE_WEDGE, "path": TT_SAMPLE_PATH}[scheme]
        buf = (Triangle * max(int(k), 1))()
        n_out = ctypes.c_uint32(0)
        st = (ctypes.c_uint64 * 2)()
        draws = np.zeros(4 * max(int(budget), 1), np.uint32) if return_draws else None
        _check(library().sample_triangles_by(self._h, sc, int(k), float(p), int(budget), int(seed) & (2**64 - 1),
                                             math.nan if q is None else float(q),
                                             None if draws is None else draws.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                             buf, ctypes.byref(n_out), ctypes.byref(st)))
        out = _result(buf, n_out.value)
        out["closed_draws"], out["distinct"] = int(st[0]), int(st[1])
        if return_draws:
            out["draws"] = draws[: 4 * int(budget)].reshape(-1, 4)
        return out

    def cliques(self, size: int, k: int, p: float, budget: int = 0, seed: int = 0, q: float | None = None,
                all_edges: bool = False):
        """Edge sampling extended to 4- or 5-cliques (Sec. 4.5): top-k cliques on the drawn edges
        (all_edges: on every edge, the exact top-k).  Returns dict(v: [n_out, size], score,
        n_out, found)."""
        buf = (Clique * max(int(k), 1))()
        n_out = ctypes.c_uint32(0)
        found = ctypes.c_uint64(0)
        _check(library().sample_heavy_cliques(self._h, int(size), int(k), float(p), int(budget),
                                              int(seed) & (2**64 - 1), math.nan if q is None else float(q),
                                              1 if all_edges else 0, buf, ctypes.byref(n_out), ctypes.byref(found)))
        nn = n_out.value
        v = np.array([list(buf[t].v)[:size] for t in range(nn)], np.uint32).reshape(nn, size)
        return {"v": v, "score": np.array([buf[t].score for t in range(nn)]), "n_out": nn, "found": int(found.value)}

    def topk_noalloc(self, k: int, p: float):
        """topk_triangles_noalloc: the same answer as topk(k, p), with no allocation."""
        buf = (Triangle * max(int(k), 1))()
        n_out = ctypes.c_uint32(0)
        _check(library().topk_triangles_noalloc(self._h, int(k), float(p), buf, ctypes.byref(n_out)))
        return _result(buf, n_out.value)

    def sample(self, k: int, p: float, budget: int, seed: int, with_stats: bool = False, q: float | None = None,
               return_draws: bool = False):
        """Weighted edge sampling (Alg. 3): top-k of the union of triangles on the drawn edges.
        q names the sampling exponent (default: p for finite p > 0, else 1); return_draws adds
        the input edge index of every draw ("draws", uint32[budget])."""
        lib = library()
        buf = (Triangle * max(int(k), 1))()
        n_out = ctypes.c_uint32(0)
        st = QueryStats()
        draws = np.zeros(max(int(budget), 1), np.uint32) if return_draws else None
        _check(lib.sample_heavy_triangles_ex(self._h, int(k), float(p), int(budget), int(seed) & (2**64 - 1),
                                             math.nan if q is None else float(q),
                                             None if draws is None else draws.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                             buf, ctypes.byref(n_out), ctypes.byref(st)))
        out = _result(buf, n_out.value)
        if with_stats:
            out["stats"] = st.as_dict()
        if return_draws:
            out["draws"] = draws[: int(budget)]
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().graph_free(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop over a resident Graph (see server_create)."""

    def __init__(self, graph: Graph, slots: int = 4, scratch_budget: int = 4 << 30):
        self.graph = graph
        self._h = ctypes.c_void_p()
        _check(library().server_create(graph.handle, int(slots), int(scratch_budget), ctypes.byref(self._h)))
        self._k = {}

    def scratch_bytes(self) -> int:
        """Device bytes the workers' scratch holds now (bounded by the budget)."""
        return int(library().server_scratch_bytes(self._h))

    def request_bytes(self, k: int, subset_n: int = 0) -> int:
        return int(library().server_request_bytes(self._h, int(k), int(subset_n)))

    def submit(self, k: int, p: float, subset=None) -> int:
        t = ctypes.c_uint64(0)
        sub_p, sub_n = None, 0
        if subset is not None and len(subset):
            sub = _u32(subset)
            sub_p, sub_n = sub.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), int(sub.shape[0])
        _check(library().server_submit(self._h, int(k), float(p), sub_p, sub_n, ctypes.byref(t)))
        self._k[t.value] = int(k)
        return int(t.value)

    def done(self, ticket: int) -> bool:
        d = ctypes.c_int(0)
        _check(library().server_poll(self._h, int(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        # the result buffer must hold the request's k: an unknown ticket never reaches the library
        k = self._k.pop(int(ticket), None)
        if k is None:
            raise ValueError(f"ticket {ticket} was not submitted here or has already been waited for")
        buf = (Triangle * max(k, 1))()
        n_out = ctypes.c_uint32(0)
        st = QueryStats()
        _check(library().server_wait(self._h, int(ticket), buf, ctypes.byref(n_out), ctypes.byref(st)))
        out = _result(buf, n_out.value)
        out["stats"] = st.as_dict()
        return out

    def info(self):
        a, c, pk = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        mq, mr = ctypes.c_uint32(), ctypes.c_uint32()
        _check(library().server_info(self._h, ctypes.byref(a), ctypes.byref(c), ctypes.byref(pk), ctypes.byref(mq),
                                     ctypes.byref(mr)))
        return {"admitted": a.value, "completed": c.value, "peak_bytes": pk.value, "max_queue": mq.value,
                "max_running": mr.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent graphs resident on the GPU, queried together (see batch_load).

    ``graphs`` is a sequence of (n, src, dst, w) with local vertex ids, or the concatenated
    form ``(ns, ms, src, dst, w)`` given through ``Batch.concat``."""

    def __init__(self, graphs=None, *, ns=None, ms=None, src=None, dst=None, w=None, stream=None):
        lib = library()
        if graphs is not None:
            graphs = list(graphs)
            ns = np.array([int(g[0]) for g in graphs], np.uint32)
            ms = np.array([len(g[1]) for g in graphs], np.uint64)
            src = np.concatenate([_u32(g[1]) for g in graphs]) if graphs else np.zeros(0, np.uint32)
            dst = np.concatenate([_u32(g[2]) for g in graphs]) if graphs else np.zeros(0, np.uint32)
            w = np.concatenate([_u32(g[3]) for g in graphs]) if graphs else np.zeros(0, np.uint32)
        ns = np.ascontiguousarray(ns, dtype=np.uint32)
        ms = np.ascontiguousarray(ms, dtype=np.uint64)
        if ns.shape != ms.shape or ns.ndim != 1:
            raise ValueError("ns and ms must be 1-D arrays of equal length")
        self._h = ctypes.c_void_p()
        p32, p64 = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
        if hasattr(src, "is_cuda") and src.is_cuda:
            import torch
            s, d, ww = (x.contiguous().to(torch.int32) for x in (src, dst, w))
            if stream is None:
                stream = torch.cuda.current_stream(src.device)
            st = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
            _check(lib.batch_load_device(len(ns), ns.ctypes.data_as(p32), ms.ctypes.data_as(p64),
                                         ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr()),
                                         ctypes.c_void_p(ww.data_ptr()), st, ctypes.byref(self._h)))
        else:
            s, d, ww = _u32(src), _u32(dst), _u32(w)
            if not (s.shape == d.shape == ww.shape) or int(ms.sum()) != s.shape[0]:
                raise ValueError("src, dst, w must hold sum(ms) edges each")
            _check(lib.batch_load(len(ns), ns.ctypes.data_as(p32), ms.ctypes.data_as(p64), s.ctypes.data_as(p32),
                                  d.ctypes.data_as(p32), ww.ctypes.data_as(p32), ctypes.byref(self._h)))
        self.count = int(len(ns))

    @staticmethod
    def num_configs() -> int:
        return int(library().batch_num_configs())

    def topk(self, k: int, p: float, config: int = -1, eager: bool = False, with_stats: bool = False):
        """Top-k of every graph.  Returns dict(i, j, l, score: [count, k] arrays (slots past
        n_out[g] are zero), n_out: [count])."""
        lib = library()
        k = int(k)
        res = np.empty(max(self.count * k, 1), TRI_DTYPE)
        n_out = np.empty(max(self.count, 1), np.uint32)
        st = BatchStats()
        _check(lib.batch_topk_ex(self._h, k, float(p), int(config), TT_BATCH_EAGER if eager else 0,
                                 ctypes.cast(res.ctypes.data, ctypes.POINTER(Triangle)),
                                 n_out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(st)))
        r = res[: self.count * k].reshape(self.count, k)
        out = {"i": r["i"], "j": r["j"], "l": r["l"], "score": r["score"], "n_out": n_out[: self.count]}
        if with_stats:
            out["stats"] = st.as_dict()
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def load(n, src, dst, w, stream=None) -> Graph:
    return Graph(n, src, dst, w, stream=stream)


def trim_cache() -> int:
    """Hands every cached device block back to the driver (tt_trim_cache); returns the bytes."""
    return int(library().tt_trim_cache())
