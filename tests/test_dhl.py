"""The paper's exact method on the CPU (Alg. 2 with alpha_p, and Auto-HL of Sec. 3.3) against
the oracle: the same answer as the plain enumeration, bit for bit at p in {-inf, 0, 1, 2, +inf}
and by the parity rule at other p, on tiny random graphs, the 2,000-node workload and (p = 1)
the 1M-vertex workload; each triangle is enumerated exactly once; validation codes."""
import itertools
import math

import numpy as np
import pytest

import graphgen
import oracle
from paritylib import EdgeIndex, assert_parity, triples
from paper_1910_00692_amd import dhl

ALL_P = [-math.inf, -3.0, -1.0, 0.0, 0.5, 1.0, 1.5, 2.0, 3.0, math.inf]


def rand_graph(rng, n, prob, whi):
    iu = np.array(list(itertools.combinations(range(n), 2)), np.uint32).reshape(-1, 2)
    e = iu[rng.random(len(iu)) < prob]
    flip = rng.random(len(e)) < 0.5
    s = np.where(flip, e[:, 1], e[:, 0]).astype(np.uint32)
    d = np.where(flip, e[:, 0], e[:, 1]).astype(np.uint32)
    return s, d, rng.integers(1, whi + 1, len(s)).astype(np.uint32)


@pytest.fixture(scope="module", autouse=True)
def built():
    from paper_1910_00692_amd._build import build_dhl
    build_dhl(force=False)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("alpha", [1.25, 0.0, 2.0])
def test_tiny_graphs_every_p(seed, alpha):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(4, 40))
    s, d, w = rand_graph(rng, n, rng.uniform(0.2, 0.8), int(rng.choice([3, 30, 10**6])))
    ei = EdgeIndex(s, d, w)
    total = oracle.count_triangles(n, s, d, w)
    for p in ALL_P:
        for k in (1, 10, 100000):
            got = dhl.topk(n, s, d, w, k, p, alpha)
            want = oracle.topk(n, s, d, w, k, p)
            assert_parity(got, want, p, ei, ctx=f"dhl tiny{seed} alpha={alpha} p={p} k={k}")
            assert got["stats"]["enumerated"] <= total
        # k beyond the count: every triangle enumerated, exactly once
        assert dhl.topk(n, s, d, w, 10**6, 1.0, alpha)["stats"]["enumerated"] == total


@pytest.mark.parametrize("p", ALL_P)
@pytest.mark.parametrize("alpha", [1.25, 0.0])
def test_small_workload(small_graph, p, alpha):
    g = small_graph
    ei = EdgeIndex(g.src, g.dst, g.w)
    for k in (1, 100, 1000, 30000):
        got = dhl.topk(g.n, g.src, g.dst, g.w, k, p, alpha)
        want = oracle.topk(g.n, g.src, g.dst, g.w, k, p)
        assert_parity(got, want, p, ei, ctx=f"dhl small alpha={alpha} p={p} k={k}")


def test_uniform_weights_pure_ties():
    n = 40
    s, d = (np.array(x, np.uint32) for x in zip(*itertools.combinations(range(n), 2)))
    w = np.full(len(s), 7, np.uint32)
    for alpha in (1.25, 0.0):
        got = dhl.topk(n, s, d, w, 500, 1.0, alpha)
        assert triples(got) == list(itertools.islice(itertools.combinations(range(n), 3), 500))


def test_medium_workload_p1_bit_exact():
    """The 1M-vertex / 20M-edge workload at p = 1, top-1000: identical to the oracle."""
    g = graphgen.medium()
    want = oracle.topk(g.n, g.src, g.dst, g.w, 1000, 1.0)
    for alpha in (1.25, 0.0):
        got = dhl.topk(g.n, g.src, g.dst, g.w, 1000, 1.0, alpha)
        for x in ("i", "j", "l", "score"):
            assert np.array_equal(got[x], want[x]), (alpha, x)
        # far fewer triangles than the 277,942,946 of the graph
        assert got["stats"]["enumerated"] < 1_000_000


def test_validation_and_arguments():
    import paper_1910_00692_amd as tt
    for n, s, d, w in ((3, [0, 1], [1, 1], [1, 1]), (3, [0, 1], [1, 0], [1, 1]), (3, [0, 1], [1, 2], [1, 0]),
                       (3, [0, 1], [1, 3], [1, 1])):
        with pytest.raises(tt.TopKError) as e:
            dhl.topk(n, s, d, w, 5, 1.0)
        assert e.value.code == oracle.validate(n, s, d, w)
    with pytest.raises(tt.TopKError):
        dhl.topk(3, [0], [1], [1], 5, 1.0, alpha=-1.0)
    assert dhl.topk(3, [0], [1], [1], 5, 1.0)["n_out"] == 0
    assert dhl.topk(5, [], [], [], 5, 1.0)["n_out"] == 0
