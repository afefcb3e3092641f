"""Edge sampling extended to 4- and 5-cliques (Sec. 4.5, Appendix A) on the GPU against the
oracle: with every edge taken (the exact top-k cliques) and with Alg. 3's draws replayed (the
same drawn edges on both sides for integer q), bit for bit at p in {-inf, 1, +inf} and by the
parity rule at other p (scores within 1e-12, set differences only at the k-th score)."""
import itertools
import math
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

EXACT = (1.0, math.inf, -math.inf)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def tt():
    import paper_1910_00692_amd as tt
    tt.library()
    return tt


def compare(got, want, p, ctx):
    assert got["n_out"] == want["n_out"], (ctx, got["n_out"], want["n_out"])
    if not got["n_out"]:
        return
    g = [tuple(v) for v in got["v"].tolist()]
    w = [tuple(v) for v in want["v"].tolist()]
    if p in EXACT:
        assert g == w, (ctx, next(t for t in range(len(g)) if g[t] != w[t]))
        assert np.array_equal(got["score"], want["score"]), ctx
        return
    np.testing.assert_allclose(got["score"], want["score"], rtol=1e-12, atol=0, err_msg=ctx)
    kth = want["score"][-1]
    sc = dict(zip(w, want["score"]))
    sc.update(zip(g, got["score"]))
    for c in set(g) ^ set(w):
        assert abs(sc[c] - kth) <= 1e-12 * kth, (ctx, c, sc[c], kth)


def graphs():
    rng = np.random.default_rng(80)
    n = 40
    iu = np.array(list(itertools.combinations(range(n), 2)), np.uint32)
    e = iu[rng.random(len(iu)) < 0.45]
    yield "random n=40", n, e[:, 0].copy(), e[:, 1].copy(), rng.integers(1, 50, len(e)).astype(np.uint32)
    g = graphgen.chung_lu(600, 6000, 2.3, 1.8, seed=81, plant=4, plant_size=5, plant_mult=1000)
    yield "chung-lu n=600 + planted K5", g.n, g.src, g.dst, g.w


@pytest.mark.parametrize("size", [4, 5])
@pytest.mark.parametrize("p", [1.0, math.inf, -math.inf, 0.5, 2.0, 0.0])
def test_exact_top_cliques(tt, size, p):
    for name, n, s, d, w in graphs():
        with tt.Graph(n, s, d, w) as G:
            for k in (1, 30, 5000):
                got = G.cliques(size, k, p, all_edges=True)
                want = oracle.cliques(n, s, d, w, size, k, p)
                compare(got, want, p, f"{name} size={size} p={p} k={k}")
                assert got["found"] == want["total"]


@pytest.mark.parametrize("size", [4, 5])
@pytest.mark.parametrize("p", [1.0, 2.0, math.inf])
def test_sampled_cliques_replay(tt, size, p):
    for name, n, s, d, w in graphs():
        with tt.Graph(n, s, d, w) as G:
            for budget, seed in ((20, 1), (500, 2), (20000, 3)):
                got = G.cliques(size, 50, p, budget=budget, seed=seed)
                want = oracle.sample_heavy_cliques(n, s, d, w, size, 50, p, budget, seed)
                compare(got, want, p, f"{name} size={size} p={p} budget={budget}")
                assert got["found"] == want["total"]
                log(f"{name} size={size} p={p} budget={budget}: {got['found']} cliques on the drawn edges")
