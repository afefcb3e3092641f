"""The static heavy-light algorithm (Alg. 1) on the GPU against its definition: the oracle's
top-k of the subgraph of the edges heavier than tau, bit for bit at the exact p and by the parity
rule elsewhere; tau = 0 is the exact answer; the fraction of the exact top-k it finds grows as
tau falls (the trade-off of Sec. 5.2, Fig. 2)."""
import math
import sys

import numpy as np
import pytest

import graphgen
import oracle
from paritylib import EdgeIndex, assert_parity

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def tt():
    import paper_1910_00692_amd as tt
    tt.library()
    return tt


def tau_for_fraction(w, f):
    """The threshold that labels about a fraction f of the edges heavy (w > tau)."""
    r = max(int(f * len(w)) - 1, 0)
    return int(np.sort(w)[::-1][r]) - 1


@pytest.mark.parametrize("p", [1.0, -math.inf, math.inf, 0.0, 2.0, 0.5])
def test_shl_is_top_k_of_heavy_subgraph(tt, p):
    g = graphgen.chung_lu(30000, 400000, 2.2, 1.8, seed=51, plant=6, plant_size=4, plant_mult=1000)
    with tt.Graph(g.n, g.src, g.dst, g.w) as G:
        for f in (0.02, 0.1, 0.5):
            tau = tau_for_fraction(g.w, f)
            heavy = g.w > tau
            got = G.shl(300, p, tau)
            assert got["heavy_edges"] == int(heavy.sum())
            want = oracle.topk(g.n, g.src[heavy], g.dst[heavy], g.w[heavy], 300, p)
            assert_parity(got, want, p, EdgeIndex(g.src[heavy], g.dst[heavy], g.w[heavy]), ctx=f"shl f={f} p={p}")
        exact = G.topk(300, p)
        every = G.shl(300, p, 0)
        assert every["n_out"] == exact["n_out"] and np.array_equal(every["i"], exact["i"])
        none = G.shl(300, p, 2**32 - 1)
        assert none["n_out"] == 0 and none["heavy_edges"] == 0


def test_shl_accuracy_grows_with_heavy_fraction(tt):
    g = graphgen.medium()
    with tt.Graph(g.n, g.src, g.dst, g.w) as G:
        exact = G.topk(1000, 1.0)
        ref = set(zip(exact["i"].tolist(), exact["j"].tolist(), exact["l"].tolist()))
        acc = []
        for f in (0.001, 0.01, 0.1, 0.5, 1.0):
            r = G.shl(1000, 1.0, tau_for_fraction(g.w, f))
            got = set(zip(r["i"].tolist(), r["j"].tolist(), r["l"].tolist()))
            acc.append(len(got & ref) / len(ref))
            log(f"shl f={f}: accuracy {acc[-1]:.3f}, {r['heavy_edges']} heavy edges")
        assert all(a <= b + 1e-12 for a, b in zip(acc, acc[1:])) and acc[-1] == 1.0
