"""Full-size parity on the 1M-vertex / 20M-edge workload (50 planted heavy 4-cliques), loaded
from device-resident tensors exactly as bench.py does, at the four p of that workload and
for edge sampling with 1e7 draws."""
import math
import sys

import numpy as np
import pytest

import graphgen
import oracle
from paritylib import EdgeIndex, assert_parity, triples

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def medium():
    import torch
    import paper_1910_00692_amd as tt
    g = graphgen.medium()
    log(f"medium n={g.n} m={g.m}")
    dev = torch.device("cuda:0")
    s = torch.from_numpy(g.src.view(np.int32)).to(dev)
    d = torch.from_numpy(g.dst.view(np.int32)).to(dev)
    w = torch.from_numpy(g.w.view(np.int32)).to(dev)
    G = tt.Graph(g.n, s, d, w, stream=torch.cuda.current_stream(dev))
    yield g, G, EdgeIndex(g.src, g.dst, g.w)
    G.close()


@pytest.mark.parametrize("p", [-math.inf, 1.0, 2.0, math.inf])
def test_medium_exact(medium, p):
    g, G, ei = medium
    log(f"medium exact p={p}")
    got = G.topk(1000, p, with_stats=True)
    want = oracle.topk(g.n, g.src, g.dst, g.w, 1000, p)
    log(f"  stats {got['stats']}")
    assert_parity(got, want, p, ei, ctx=f"medium p={p}")
    # every planted 4-clique triangle has all weights >= 1000; at p = -inf they outrank all
    # natural triangles whose lightest edge is below 1000
    if p == -math.inf:
        planted = set()
        for c in g.planted.tolist():
            c = sorted(c)
            planted |= {(c[0], c[1], c[2]), (c[0], c[1], c[3]), (c[0], c[2], c[3]), (c[1], c[2], c[3])}
        assert planted <= set(triples(got))


@pytest.mark.parametrize("p", [-math.inf, 1.0, 2.0, math.inf, 3.0])
def test_medium_sampling(medium, p):
    """Edge sampling with 1e7 draws at every p of the workload (q = 1 for p = +-inf, q = 2 at
    p = 2: the 128-bit prefix scan, guide table and draw at m = 20M), and at p = 3, where this
    graph's weights give Z = sum w^3 > 2^64, so the draw target's high term is exercised."""
    g, G, ei = medium
    log(f"medium sampling p={p}")
    got = G.sample(1000, p, 10_000_000, seed=1234, with_stats=True)
    want = oracle.sample_heavy_triangles(g.n, g.src, g.dst, g.w, 1000, p, 10_000_000, 1234)
    log(f"  stats {got['stats']}")
    if p == 3.0:
        assert sum(int(x) ** 3 for x in np.sort(g.w)[-200000:].tolist()) >= 2**64
    assert got["stats"]["distinct_sampled"] == want["distinct_edges"]
    assert_parity(got, want, p, ei, ctx=f"medium es p={p}")


def test_medium_subset_with_hubs(medium):
    """A subset holding the 50 highest-degree vertices: their in-neighbours' rows hold far more
    entries than the compact stream, most of which are dropped, so the stream is built from a
    scan of those rows (and used if what is kept fits).  Against the oracle."""
    g, G, ei = medium
    deg = np.bincount(g.src, minlength=g.n) + np.bincount(g.dst, minlength=g.n)
    hubs = np.argsort(deg)[-50:]
    rng = np.random.default_rng(77)
    sub = np.unique(np.concatenate([hubs, rng.choice(g.n, size=950, replace=False)])).astype(np.uint32)
    for p in (1.0, -math.inf):
        got = G.topk(500, p, subset=sub, with_stats=True)
        log(f"  hubs p={p} stats {got['stats']}")
        vm = np.zeros(g.n, np.uint8)
        vm[sub.astype(np.int64)] = 1
        want = oracle.topk(g.n, g.src, g.dst, g.w, 500, p, vertex_mark=vm)
        assert_parity(got, want, p, ei, ctx=f"medium subset with hubs p={p}")


@pytest.mark.parametrize("size,p", [(1000, 1.0), (1000, 0.0), (300_000, 2.0)])
def test_medium_subset(medium, size, p):
    """A 1,000-vertex subset takes the compact stream of its possible base entries; a
    300,000-vertex subset has more such entries than that stream holds and streams every
    entry with the vertex pre-tests instead.  Both against the oracle."""
    g, G, ei = medium
    rng = np.random.default_rng(size)
    sub = rng.choice(g.n, size=size, replace=False).astype(np.uint32)
    log(f"medium subset size={size} p={p}")
    got = G.topk(500, p, subset=sub, with_stats=True)
    log(f"  stats {got['stats']}")
    vm = np.zeros(g.n, np.uint8)
    vm[sub.astype(np.int64)] = 1
    want = oracle.topk(g.n, g.src, g.dst, g.w, 500, p, vertex_mark=vm)
    assert_parity(got, want, p, ei, ctx=f"medium subset={size} p={p}")
    if size == 1000:
        assert got["stats"]["edges_streamed"] < g.m  # the compact stream, not the graph
