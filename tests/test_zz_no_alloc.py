"""topk_triangles_noalloc (the entry point for callers that cannot allocate) against
topk_triangles, called through the C ABI: two calls in a row, the second on a smaller graph
with a smaller k (the static scratch keeps the first call's contents), every kind of p, a
query whose triangle buffer overflows the fixed region (restarts above the k-th key), and the
size limit."""
import ctypes
import itertools
import math
import sys

import numpy as np
import pytest

import graphgen
from paritylib import EdgeIndex, assert_parity, triples

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def tt():
    import paper_1910_00692_amd as tt
    tt.library()
    return tt


def noalloc(tt, G, k, p):
    lib = tt.library()
    buf = (tt.Triangle * max(k, 1))()
    n_out = ctypes.c_uint32(0)
    rc = lib.topk_triangles_noalloc(G.handle, k, p, buf, ctypes.byref(n_out))
    if rc != tt.TT_OK:
        raise tt.TopKError(rc, lib.tt_last_error().decode())
    return tt._result(buf, n_out.value)


def same(a, b):
    return a["n_out"] == b["n_out"] and triples(a) == triples(b) and np.array_equal(a["score"], b["score"])


def test_noalloc_equals_topk_two_calls(tt):
    big = graphgen.chung_lu(60000, 700000, 2.1, 1.8, seed=41, plant=5, plant_size=4, plant_mult=1000)
    small = graphgen.chung_lu(2500, 25000, 2.4, 2.0, seed=42)
    for p in (1.0, -math.inf, math.inf, 0.0, 2.0, 0.5, -1.0):
        with tt.Graph(big.n, big.src, big.dst, big.w) as G1, tt.Graph(small.n, small.src, small.dst, small.w) as G2:
            for G, g, k in ((G1, big, 8000), (G2, small, 300)):
                before = G.device_bytes
                a = noalloc(tt, G, k, p)
                assert G.device_bytes == before  # nothing of the graph was built for it
                b = G.topk(k, p)
                log(f"p={p} m={g.m} k={k}: {a['n_out']} triangles")
                if p in (1.0, -math.inf, math.inf, 0.0, 2.0):
                    assert same(a, b), (p, g.m, k)
                else:
                    assert_parity(a, b, p, EdgeIndex(g.src, g.dst, g.w), ctx=f"noalloc p={p} m={g.m}")


def test_noalloc_after_orders_and_streams_exist(tt):
    """Once topk_triangles has placed the weight-ordered stream and built a bound order, the
    no-allocation call streams them too; answers stay the same."""
    g = graphgen.chung_lu(20000, 200000, 2.2, 1.8, seed=43)
    with tt.Graph(g.n, g.src, g.dst, g.w) as G:
        for rep in range(30):
            r = G.topk(500, 1.0, with_stats=True)
            if r["stats"]["bound_order"]:
                break
        G.topk(500, -math.inf)
        for p in (1.0, -math.inf):
            assert same(noalloc(tt, G, 500, p), G.topk(500, p))


def test_noalloc_overflow_restarts_and_limits(tt):
    n = 300
    s, d = (np.array(x, np.uint32) for x in zip(*itertools.combinations(range(n), 2)))
    with tt.Graph(n, s, d, np.full(len(s), 5, np.uint32)) as G:
        for k in (100, 16384):
            a = noalloc(tt, G, k, 1.0)
            assert triples(a) == list(itertools.islice(itertools.combinations(range(n), 3), k))
        with pytest.raises(tt.TopKError) as e:
            noalloc(tt, G, 16385, 1.0)
        assert e.value.code == tt.TT_E_TOO_LARGE
        assert noalloc(tt, G, 0, 1.0)["n_out"] == 0
