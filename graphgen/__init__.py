"""Seeded synthetic inputs (edge lists, weights, query streams).

This module holds no part of the method's arithmetic: it only produces graphs and query
parameters that both the CPU oracle and the GPU library consume.  The native part
(``graphgen.c``) is compiled with gcc into ``libgraphgen.so`` next to this file.

Workload recipes (the paper's datasets are not available; these stand in for them, with
power-law degrees like the configuration model of Sec. 3.3 and heavy-tailed Zipf weights
like Fig. 1):

* ``small``   : Chung-Lu, n=2,000, ~20,000 edges, gamma 2.5, Zipf(s=2) on [1, 1e6], seed 0.
* ``medium``  : Chung-Lu, n=1M, ~20M edges, gamma 2.1, Zipf(s=1.8), plus 50 planted
                4-cliques whose weights are multiplied by 1000, seed 0.
* ``large``   : Chung-Lu, n=100M, ~2B edges, gamma 2.0, Zipf(s=1.5), seed 0.
* ``batch``   : 4096 independent Chung-Lu graphs, n log-uniform in [50, 20000], average
                degree uniform in [4, 40], gamma 2.5, Zipf(s=2).
* ``serve``   : Chung-Lu, n=10M, ~200M edges, gamma 2.1, Zipf(s=1.8), and a Poisson query
                stream (see :func:`query_stream`).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

GG_OK, GG_E_ARG, GG_E_NOMEM, GG_E_CAPACITY = 0, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, u32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        p32 = ctypes.POINTER(ctypes.c_uint32)
        p64 = ctypes.POINTER(ctypes.c_uint64)
        lib.gg_chung_lu.argtypes = [u64, u64, dbl, dbl, u32, u64, u64, p32, p32, p32, p64]
        lib.gg_chung_lu.restype = ctypes.c_int
        lib.gg_plant_cliques.argtypes = [u64, p64, u64, p32, p32, p32, u32, u32, u32, dbl, u32, u64, p32]
        lib.gg_plant_cliques.restype = ctypes.c_int
        lib.gg_zipf.argtypes = [u64, dbl, u32, u64, p32]
        lib.gg_zipf.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


class Graph:
    """An undirected weighted edge list: ``src``, ``dst``, ``w`` are uint32 arrays of length m."""

    def __init__(self, n: int, src: np.ndarray, dst: np.ndarray, w: np.ndarray, planted=None, name=""):
        self.n = int(n)
        self.src = src
        self.dst = dst
        self.w = w
        self.planted = planted
        self.name = name

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def __repr__(self):
        return f"Graph({self.name!r}, n={self.n}, m={self.m})"


def chung_lu(n: int, m: int, gamma: float, zipf_s: float, seed: int = 0, wmax: int = 10**6,
             plant: int = 0, plant_size: int = 4, plant_mult: int = 1000, name: str = "") -> Graph:
    """Weighted Chung-Lu graph (expected ~m edges) with optional planted heavy cliques."""
    lib = _load()
    extra = plant * plant_size * (plant_size - 1) // 2
    cap = int(m * 1.02 + 10 * math.sqrt(m) + 1024) + extra
    src = np.empty(cap, np.uint32)
    dst = np.empty(cap, np.uint32)
    w = np.empty(cap, np.uint32)
    mo = ctypes.c_uint64(0)
    rc = lib.gg_chung_lu(n, m, float(gamma), float(zipf_s), wmax, seed & (2**64 - 1), cap,
                         _p32(src), _p32(dst), _p32(w), ctypes.byref(mo))
    if rc != GG_OK:
        raise RuntimeError(f"gg_chung_lu failed: {rc}")
    planted = None
    if plant:
        members = np.empty(plant * plant_size, np.uint32)
        rc = lib.gg_plant_cliques(n, ctypes.byref(mo), cap, _p32(src), _p32(dst), _p32(w), plant, plant_size,
                                  plant_mult, float(zipf_s), wmax, seed & (2**64 - 1), _p32(members))
        if rc != GG_OK:
            raise RuntimeError(f"gg_plant_cliques failed: {rc}")
        planted = members.reshape(plant, plant_size)
    k = int(mo.value)
    return Graph(n, src[:k], dst[:k], w[:k], planted=planted, name=name)


def zipf(count: int, s: float, wmax: int = 10**6, seed: int = 0) -> np.ndarray:
    """Zipf(s) draws truncated to [1, wmax]."""
    out = np.empty(count, np.uint32)
    rc = _load().gg_zipf(count, float(s), wmax, seed, _p32(out))
    if rc != GG_OK:
        raise RuntimeError(f"gg_zipf failed: {rc}")
    return out


# ----------------------------------------------------------------------------- named workloads

def small(seed: int = 0) -> Graph:
    """n=2,000, ~20,000 edges, gamma 2.5, Zipf(s=2) weights on [1, 1e6]."""
    return chung_lu(2000, 20000, 2.5, 2.0, seed=seed, name="chung-lu n=2k m~20k g2.5 zipf2")


def medium(seed: int = 0, n: int = 1_000_000, m: int = 20_000_000) -> Graph:
    """n=1M, ~20M edges, gamma 2.1, Zipf(s=1.8), 50 planted 4-cliques with weights x1000."""
    return chung_lu(n, m, 2.1, 1.8, seed=seed, plant=50, plant_size=4, plant_mult=1000,
                    name=f"chung-lu n={n} m~{m} g2.1 zipf1.8 +50 planted K4 x1000")


def large(seed: int = 0, n: int = 100_000_000, m: int = 2_000_000_000) -> Graph:
    """n=100M, ~2B edges, gamma 2.0, Zipf(s=1.5)."""
    return chung_lu(n, m, 2.0, 1.5, seed=seed, name=f"chung-lu n={n} m~{m} g2.0 zipf1.5")


def serve_graph(seed: int = 0, n: int = 10_000_000, m: int = 200_000_000) -> Graph:
    """n=10M, ~200M edges, gamma 2.1, Zipf(s=1.8)."""
    return chung_lu(n, m, 2.1, 1.8, seed=seed, name=f"chung-lu n={n} m~{m} g2.1 zipf1.8")


def batch_specs(count: int = 4096, seed: int = 0, n_lo: int = 50, n_hi: int = 20000,
                d_lo: float = 4.0, d_hi: float = 40.0):
    """(n, m, seed) for each graph of the batched workload: n log-uniform, degree uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count)).astype(np.int64)
    ds = rng.uniform(d_lo, d_hi, count)
    ms = np.maximum(1, np.round(ns * ds / 2.0)).astype(np.int64)
    seeds = rng.integers(0, 2**62, count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(ns, ms, seeds)]


def batch(count: int = 4096, seed: int = 0, workers: int = 0, **kw):
    """The batched workload: a list of independent Chung-Lu graphs (gamma 2.5, Zipf(s=2)).

    Graphs are generated on a thread pool (the C generator releases the GIL); each graph has its
    own seed, so the result does not depend on the number of workers."""
    from concurrent.futures import ThreadPoolExecutor
    specs = batch_specs(count, seed, **kw)
    workers = workers or min(16, os.cpu_count() or 1)

    def one(i):
        n, m, s = specs[i]
        return chung_lu(n, m, 2.5, 2.0, seed=s, name=f"batch[{i}]")

    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, range(len(specs))))


P_CHOICES = (-math.inf, -1.0, 0.0, 1.0, 2.0, math.inf)


def query_stream(count: int, n: int, seed: int = 0, rate_hz: float = 2000.0, k_lo: int = 10,
                 k_hi: int = 10_000, subset_frac: float = 0.2, subset_size: int = 1000):
    """Poisson query stream: arrival time (s), k log-uniform, p from P_CHOICES, optional subset."""
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5E5E))
    gaps = rng.exponential(1.0 / rate_hz, count)
    t = np.cumsum(gaps) - gaps[0]
    ks = np.floor(np.exp(rng.uniform(math.log(k_lo), math.log(k_hi), count))).astype(np.int64)
    ps = rng.integers(0, len(P_CHOICES), count)
    sub = rng.random(count) < subset_frac
    out = []
    for i in range(count):
        subset = None
        if sub[i]:
            subset = np.sort(rng.choice(n, size=subset_size, replace=False)).astype(np.uint32)
        out.append({"t": float(t[i]), "k": int(ks[i]), "p": float(P_CHOICES[ps[i]]), "subset": subset})
    return out
