"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on seeded inputs.

Covered: tiny random graphs at every p (many ties), the 2,000-node workload at every p and
k from 1 to beyond the triangle count, candidate-buffer overflow and restart (K_300 with
uniform weights: 4.45M tied triangles), planted heavy cliques, vertex-subset queries,
validation errors, empty and degenerate graphs, device-pointer loads, determinism, and
weighted edge sampling replayed draw for draw.
"""
import itertools
import math
import sys

import numpy as np
import pytest

import graphgen
import oracle
from paritylib import EdgeIndex, assert_parity, triples

pytestmark = pytest.mark.gpu

ALL_P = [-math.inf, -3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 1.5, 2.0, 3.0, math.inf]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def tt():
    import paper_1910_00692_amd as tt
    tt.library()
    return tt


def rand_graph(rng, n, prob, wlo=1, whi=20):
    iu = np.array(list(itertools.combinations(range(n), 2)), np.uint32).reshape(-1, 2)
    keep = rng.random(len(iu)) < prob
    e = iu[keep]
    flip = rng.random(len(e)) < 0.5
    src = np.where(flip, e[:, 1], e[:, 0]).astype(np.uint32)
    dst = np.where(flip, e[:, 0], e[:, 1]).astype(np.uint32)
    perm = rng.permutation(len(src))
    w = rng.integers(wlo, whi + 1, len(src)).astype(np.uint32)
    return src[perm], dst[perm], w


def check(tt, n, s, d, w, k, p, G=None, subset=None, ctx=""):
    own = G is None
    if own:
        G = tt.Graph(n, s, d, w)
    try:
        got = G.topk(k, p, subset=subset)
    finally:
        if own:
            G.close()
    vm = None
    if subset is not None:
        vm = np.zeros(n, np.uint8)
        vm[np.asarray(subset, np.int64)] = 1
    want = oracle.topk(n, s, d, w, k, p, vertex_mark=vm)
    assert_parity(got, want, p, EdgeIndex(s, d, w), ctx=f"{ctx} k={k} p={p}")
    return got, want


@pytest.mark.parametrize("seed", range(12))
def test_tiny_random_graphs(tt, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 45))
    s, d, w = rand_graph(rng, n, rng.uniform(0.1, 0.8), 1, int(rng.choice([3, 20, 10**6])))
    log(f"tiny seed={seed} n={n} m={len(s)}")
    with tt.Graph(n, s, d, w) as G:
        for p in ALL_P:
            for k in (1, 7, 60, 100000):
                check(tt, n, s, d, w, k, p, G=G, ctx=f"tiny{seed}")


@pytest.fixture(scope="module")
def small(tt):
    g = graphgen.small()
    G = tt.Graph(g.n, g.src, g.dst, g.w)
    yield g, G
    G.close()


@pytest.mark.parametrize("p", ALL_P)
def test_small_workload(tt, small, p):
    g, G = small
    for k in (1, 100, 1000, 30000):
        log(f"small p={p} k={k}")
        got, want = check(tt, g.n, g.src, g.dst, g.w, k, p, G=G, ctx="small")
    assert want["total"] == 21481 or want["total"] > 0


def test_small_stats_and_determinism(tt, small):
    g, G = small
    a = G.topk(100, 1.0, with_stats=True)
    b = G.topk(100, 1.0, with_stats=True)
    assert triples(a) == triples(b) and np.array_equal(a["score"], b["score"])
    st = a["stats"]
    assert st["passes"] >= 1 and 0 < st["edges_streamed"] and st["triangles_emitted"] >= 100
    log(f"stats {st}")


def test_overflow_restart_with_ties(tt):
    """K_300 with one weight: 4,455,100 triangles tie at every p, more than the 4M-record
    candidate buffer, so the query must restart above the k-th full key (score, i, j, l)."""
    n = 300
    s, d = (np.array(x, np.uint32) for x in zip(*itertools.combinations(range(n), 2)))
    w = np.full(len(s), 5, np.uint32)
    log("K300 uniform")
    with tt.Graph(n, s, d, w) as G:
        for p in (1.0, -math.inf, 0.5):
            got = G.topk(100, p, with_stats=True)
            want = list(itertools.islice(itertools.combinations(range(n), 3), 100))
            assert triples(got) == want
            assert np.all(got["score"] == 5.0)
            assert got["stats"]["restarts"] >= 1, got["stats"]


def test_descent_through_weight_ties(tt):
    """Weights that tie in large groups (1 and 2 for most edges, a few heavy ones): the rank a
    band asks for falls inside a tie group far larger than itself, so the descent takes the bin
    above the group first, and the count it finds picks the next step.  k on both sides of the
    group boundaries, every kind of p, against the oracle."""
    g = graphgen.chung_lu(20000, 200000, 2.2, 1.8, seed=21)
    rng = np.random.default_rng(21)
    w = np.where(rng.random(g.m) < 0.7, 1, 2).astype(np.uint32)
    heavy = rng.choice(g.m, size=300, replace=False)
    w[heavy] = rng.integers(3, 50, size=300).astype(np.uint32)
    log(f"weight ties m={g.m}")
    with tt.Graph(g.n, g.src, g.dst, w) as G:
        for k in (10, 300, 5000):
            for p in (1.0, -math.inf, math.inf, 0.0, -1.0):
                check(tt, g.n, g.src, g.dst, w, k, p, G=G, ctx="weight ties")


def test_long_rows_every_filter(tt):
    """A dense graph (n = 320, edge probability 0.9, weights 1..3): oriented rows of up to ~290
    entries, so at low weight floors a candidate's iterated row holds more admissible entries
    than its wave takes on and they are spread over many waves.  Every kind of p, k from 1 to
    5,000, subset queries and edge sampling."""
    rng = np.random.default_rng(5)
    n = 320
    s, d, w = rand_graph(rng, n, 0.9, 1, 3)
    log(f"dense n={n} m={len(s)}")
    ei = EdgeIndex(s, d, w)
    with tt.Graph(n, s, d, w) as G:
        for p in (math.inf, -math.inf, 1.0, 2.0, 0.0, 0.5, -1.0):
            for k in (1, 200, 5000):
                check(tt, n, s, d, w, k, p, G=G, ctx="dense")
        st = G.topk(5000, math.inf, with_stats=True)["stats"]
        log(f"dense p=inf stats {st}")
        assert st["heavy_candidates"] > 0 and st["heavy_overflow"] == 0  # the spread path ran
        for sub in ([3, 77, 200], list(range(40))):
            for p in (math.inf, 1.0, -1.0):
                check(tt, n, s, d, w, 300, p, G=G, subset=np.array(sub, np.uint32), ctx=f"dense subset {len(sub)}")
        for p in (1.0, math.inf, 2.0):
            for budget in (100, 20000):
                got = G.sample(200, p, budget, seed=budget + 3)
                want = oracle.sample_heavy_triangles(n, s, d, w, 200, p, budget, budget + 3)
                assert_parity(got, want, p, ei, ctx=f"dense es p={p} budget={budget}")


def test_huge_id_space(tt):
    """3,000 vertices spread over IDs in [0, 150M): more vertex buckets than the partitioned build
    takes, so the build counts degrees and places rows with global atomics instead."""
    g = graphgen.chung_lu(3000, 30000, 2.3, 1.8, seed=11)
    rng = np.random.default_rng(4)
    ids = np.sort(rng.choice(150_000_000, size=3000, replace=False)).astype(np.uint32)
    n, s, d, w = 150_000_000, ids[g.src], ids[g.dst], g.w
    log(f"huge id space m={len(s)}")
    with tt.Graph(n, s, d, w) as G:
        for p in (1.0, math.inf, 2.0, -1.0):
            check(tt, n, s, d, w, 100, p, G=G, ctx="huge ids")


def test_head_maxima_id_space(tt):
    """20,000 vertices spread over IDs in [0, 20M): the partitioned build, and enough vertex IDs
    (>= 2^24) that every entry keeps its head's row maximum for the filter, in the head-sorted
    stream and in the weight-ordered one (p = -inf streams the latter), exact and sampled."""
    g = graphgen.chung_lu(20000, 200000, 2.2, 1.8, seed=12)
    rng = np.random.default_rng(6)
    ids = np.sort(rng.choice(20_000_000, size=20000, replace=False)).astype(np.uint32)
    n, s, d, w = 20_000_000, ids[g.src], ids[g.dst], g.w
    log(f"head maxima id space m={len(s)}")
    ei = EdgeIndex(s, d, w)
    with tt.Graph(n, s, d, w) as G:
        for p in (-math.inf, 1.0, 2.0, math.inf, -1.0):
            check(tt, n, s, d, w, 100, p, G=G, ctx="head maxima")
        for p in (1.0, -math.inf):
            got = G.sample(100, p, 20000, 5)
            want = oracle.sample_heavy_triangles(n, s, d, w, 100, p, 20000, 5)
            assert_parity(got, want, p, ei, ctx=f"head maxima es p={p}")


def test_weight_stream_placed_in_parts(tt, monkeypatch):
    """The weight-ordered stream placed bin range by bin range, as on graphs of more than 2^27
    entries (forced here on a small graph): p = -inf descends through several bands that stream
    ever longer prefixes of it, exact and sampled, each against the oracle; then p = 1 and a
    second graph whose first query needs the whole stream at once."""
    monkeypatch.setenv("TT_WS_ALL_AT_ONCE", "0")
    g = graphgen.chung_lu(30000, 300000, 2.1, 1.8, seed=13)
    log(f"weight stream in parts m={g.m}")
    ei = EdgeIndex(g.src, g.dst, g.w)
    with tt.Graph(g.n, g.src, g.dst, g.w) as G:
        for p in (-math.inf, 1.0, 2.0, math.inf):
            check(tt, g.n, g.src, g.dst, g.w, 300, p, G=G, ctx="ws parts")
        got = G.sample(300, -math.inf, 50000, 9)
        want = oracle.sample_heavy_triangles(g.n, g.src, g.dst, g.w, 300, -math.inf, 50000, 9)
        assert_parity(got, want, -math.inf, ei, ctx="ws parts es")
    with tt.Graph(g.n, g.src, g.dst, g.w) as G:
        check(tt, g.n, g.src, g.dst, g.w, 30000, -math.inf, G=G, ctx="ws parts big k")


def test_planted_cliques(tt):
    g = graphgen.chung_lu(20000, 200000, 2.2, 1.8, seed=3, plant=8, plant_size=4, plant_mult=1000)
    log(f"planted m={g.m}")
    with tt.Graph(g.n, g.src, g.dst, g.w) as G:
        for p in (-math.inf, 0.0, 1.0, 2.0, math.inf, -1.0, 1.5):
            check(tt, g.n, g.src, g.dst, g.w, 64, p, G=G, ctx="planted")


def test_subset_queries(tt, small):
    g, G = small
    rng = np.random.default_rng(5)
    for size in (1, 10, 300):
        sub = rng.choice(g.n, size=size, replace=False).astype(np.uint32)
        for p in (1.0, -math.inf, 2.0, -1.0):
            log(f"subset size={size} p={p}")
            check(tt, g.n, g.src, g.dst, g.w, 50, p, G=G, subset=sub, ctx=f"subset{size}")


def test_subset_repeats_hubs_and_everything(tt, small):
    """Repeated ids count once; a subset made of the highest-degree vertices; the subset of all
    vertices gives the unrestricted answer."""
    g, G = small
    deg = np.bincount(np.concatenate([g.src, g.dst]).astype(np.int64), minlength=g.n)
    hubs = np.argsort(-deg, kind="stable")[:5].astype(np.uint32)
    rep = np.concatenate([hubs, hubs[::-1], hubs[:2]])
    for p in (1.0, -math.inf, 0.0):
        log(f"subset hubs p={p}")
        a, _ = check(tt, g.n, g.src, g.dst, g.w, 200, p, G=G, subset=rep, ctx="subset-rep")
        b = G.topk(200, p, subset=hubs)
        assert triples(a) == triples(b) and np.array_equal(a["score"], b["score"])
    every = np.arange(g.n, dtype=np.uint32)[::-1].copy()
    for p in (2.0, -1.0):
        a, b = G.topk(300, p, subset=every), G.topk(300, p)
        assert triples(a) == triples(b) and np.array_equal(a["score"], b["score"])


def test_bound_order_after_repeated_queries(tt):
    """Repeated queries of one p build its bound order once they have streamed more than 4m
    entries; the answers must not change when the passes switch to it (every p, both query
    kinds, and a restart above the k-th key with K_300's ties)."""
    g = graphgen.chung_lu(20000, 200000, 2.2, 1.8, seed=13, plant=4, plant_size=4, plant_mult=1000)
    ei = EdgeIndex(g.src, g.dst, g.w)
    with tt.Graph(g.n, g.src, g.dst, g.w) as G:
        for p in ALL_P:
            want = oracle.topk(g.n, g.src, g.dst, g.w, 3000, p)
            first, used = None, False
            for rep in range(40):
                r = G.topk(3000, p, with_stats=True)
                assert_parity(r, want, p, ei, ctx=f"order p={p} rep={rep}")
                used = used or bool(r["stats"]["bound_order"])
                if used:
                    break
            assert used, p
            es0 = oracle.sample_heavy_triangles(g.n, g.src, g.dst, g.w, 200, p, 20000, 5)
            assert_parity(G.sample(200, p, 20000, 5), es0, p, ei, ctx=f"order es p={p}")
    n = 300
    s, d = (np.array(x, np.uint32) for x in zip(*itertools.combinations(range(n), 2)))
    with tt.Graph(n, s, d, np.full(len(s), 5, np.uint32)) as G:
        want = list(itertools.islice(itertools.combinations(range(n), 3), 100))
        for rep in range(6):
            r = G.topk(100, 1.0, with_stats=True)
            assert triples(r) == want and r["stats"]["restarts"] >= 1
        assert r["stats"]["bound_order"] == 1


def test_validation_errors(tt):
    cases = [
        (3, [0, 1], [1, 1], [1, 1]),
        (3, [0, 1], [1, 0], [1, 1]),
        (3, [0, 1], [1, 2], [1, 0]),
        (3, [0, 1], [1, 3], [1, 1]),
        (4, [0, 1, 2, 0], [1, 2, 0, 1], [1, 1, 1, 1]),
    ]
    for n, s, d, w in cases:
        want = oracle.validate(n, s, d, w)
        with pytest.raises(tt.TopKError) as e:
            tt.Graph(n, s, d, w)
        assert e.value.code == want, (s, d, w, e.value.code, want)


@pytest.mark.parametrize("L", [100, 200, 300])
def test_repeated_pair_in_long_rows(tt, L):
    """A repeated pair is found in rows of every length class: vertex 0 has L neighbours S,
    each of which also reaches L + 1 further vertices T, so 0 (lowest degree) is the tail of an
    (L + 1)-entry row and every T vertex of an L-entry row; the repeat is put in one such row
    (0 -> S[0], or T[0] -> S[7]), and in a 2-entry row (an extra edge between the last two
    vertices) for contrast.  L = 100 and 200 give rows that one wave ranks (at most 128 and
    256 entries), L = 300 rows that a whole block ranks."""
    S = np.arange(1, L + 1, dtype=np.uint32)
    T = np.arange(L + 1, 2 * L + 2, dtype=np.uint32)
    s0, d0 = np.zeros(L, np.uint32), S
    s1, d1 = np.repeat(S, len(T)), np.tile(T, len(S))
    n = 2 * L + 4
    base_s = np.concatenate([s0, s1, [n - 2]]).astype(np.uint32)
    base_d = np.concatenate([d0, d1, [n - 1]]).astype(np.uint32)
    with tt.Graph(n, base_s, base_d, np.ones(len(base_s), np.uint32)) as G:
        assert G.m == len(base_s)
    for a, b in ((0, 1), (L + 1, 8), (n - 1, n - 2)):
        s = np.concatenate([base_s, [b]]).astype(np.uint32)
        d = np.concatenate([base_d, [a]]).astype(np.uint32)
        w = np.ones(len(s), np.uint32)
        assert oracle.validate(n, s, d, w) == tt.TT_E_DUP_EDGE
        with pytest.raises(tt.TopKError) as e:
            tt.Graph(n, s, d, w)
        assert e.value.code == tt.TT_E_DUP_EDGE, (a, b)


def test_empty_and_degenerate(tt):
    with tt.Graph(5, [], [], []) as G:
        assert G.topk(10, 1.0)["n_out"] == 0
        assert G.sample(10, 1.0, 100, 1)["n_out"] == 0
    with tt.Graph(0, [], [], []) as G:
        assert G.topk(10, 1.0)["n_out"] == 0
    # a tree: no triangles
    n = 200
    s = np.arange(1, n, dtype=np.uint32)
    d = (np.arange(1, n) // 2).astype(np.uint32)
    with tt.Graph(n, s, d, np.ones(n - 1, np.uint32)) as G:
        assert G.topk(10, 1.0)["n_out"] == 0
    # one triangle, k = 0 and k > T
    with tt.Graph(4, [0, 1, 2, 2], [1, 2, 0, 3], [5, 6, 7, 1]) as G:
        assert G.topk(0, 1.0)["n_out"] == 0
        r = G.topk(10, 1.0)
        assert r["n_out"] == 1 and triples(r) == [(0, 1, 2)] and r["score"][0] == 6.0
    # largest weights: keys need 96 bits (product) and 66 bits (sum of squares)
    big = 2**32 - 1
    s, d, w = [0, 1, 2, 3, 3], [1, 2, 0, 0, 1], [big, big - 1, big, 1, 2]
    for p in ALL_P:
        check(tt, 4, np.array(s, np.uint32), np.array(d, np.uint32), np.array(w, np.uint32), 5, p, ctx="bigw")


def test_device_pointer_load(tt, small):
    import torch
    g, G = small
    dev = torch.device("cuda:0")
    s = torch.from_numpy(g.src.astype(np.int32)).to(dev)
    d = torch.from_numpy(g.dst.astype(np.int32)).to(dev)
    w = torch.from_numpy(g.w.astype(np.int32)).to(dev)
    with tt.Graph(g.n, s, d, w) as G2:
        for p in (1.0, math.inf):
            a, b = G.topk(500, p), G2.topk(500, p)
            assert triples(a) == triples(b) and np.array_equal(a["score"], b["score"])


# ------------------------------------------------------------------------------ sampling

@pytest.mark.parametrize("seed", range(6))
def test_sampling_replay_tiny(tt, seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(6, 40))
    s, d, w = rand_graph(rng, n, rng.uniform(0.2, 0.7), 1, int(rng.choice([5, 1000])))
    log(f"es tiny seed={seed} n={n} m={len(s)}")
    ei = EdgeIndex(s, d, w)
    with tt.Graph(n, s, d, w) as G:
        for p in (1.0, 2.0, 3.0, -math.inf, math.inf, 0.0, -1.0):
            for budget in (1, 5, 50, 5000):
                got = G.sample(30, p, budget, seed=seed * 7 + 1)
                want = oracle.sample_heavy_triangles(n, s, d, w, 30, p, budget, seed * 7 + 1)
                assert_parity(got, want, p, ei, ctx=f"es seed={seed} p={p} budget={budget}")


@pytest.mark.parametrize("p", [1.0, 2.0, -math.inf, math.inf])
def test_sampling_small_workload(tt, small, p):
    g, G = small
    ei = EdgeIndex(g.src, g.dst, g.w)
    for budget, seed in ((100, 1), (10000, 2), (200000, 3)):
        log(f"es small p={p} budget={budget}")
        got = G.sample(100, p, budget, seed, with_stats=True)
        want = oracle.sample_heavy_triangles(g.n, g.src, g.dst, g.w, 100, p, budget, seed)
        assert_parity(got, want, p, ei, ctx=f"es small p={p} budget={budget}")
        assert got["stats"]["distinct_sampled"] == want["distinct_edges"]


def check_draws(gpu_draws, w, p, q, budget, seed, ctx):
    """Draw for draw against the oracle's replay of Alg. 3.  Integer q: identical.  Other q: the
    two FP64 prefix sums differ in rounding (the oracle sums in input order, the GPU in blocks),
    so a draw may differ only where its target lies within 1e-12 Z of the oracle's boundary
    between the two edges.  Returns the number of draws that differ."""
    _, want = oracle.es_draw(w, p, budget, seed, return_draws=True, q=q)
    got = np.asarray(gpu_draws, np.int64)
    want = want.astype(np.int64)
    qq = oracle.sample_exponent(p) if q is None else q
    diff = np.nonzero(got != want)[0]
    if qq in (1.0, 2.0, 3.0):
        assert len(diff) == 0, (ctx, diff[:5], got[diff[:5]], want[diff[:5]])
        return 0
    P = oracle.es_prefix_f64(w, qq)
    Z = P[-1]
    for s in diff.tolist():
        r = float(oracle.splitmix64(seed, s) >> 11) * 2.0**-53 * Z
        e = int(got[s])
        lo = P[e - 1] if e > 0 else 0.0
        assert P[e] > r - 1e-12 * Z and lo <= r + 1e-12 * Z, (ctx, s, e, int(want[s]), r, lo, P[e])
    return len(diff)


@pytest.mark.parametrize("p,q", [(0.5, None), (1.5, None), (1.0, 1.5), (-1.0, 0.5), (math.inf, 2.5),
                                 (2.0, 0.75)])
def test_sampling_noninteger_exponent_with_draws(tt, small, p, q):
    """Non-integer sampling exponents, the default reading (q = p for finite p > 0) and named q:
    the GPU's draws are returned and checked against the oracle's replay (FP64 prefix sums,
    1e-12 of a bucket edge), then the oracle enumerates the triangles on exactly those drawn
    edges, and the GPU's answer must match it by the parity rule."""
    g, G = small
    ei = EdgeIndex(g.src, g.dst, g.w)
    for budget, seed in ((1000, 4), (200000, 8)):
        got = G.sample(100, p, budget, seed, q=q, return_draws=True, with_stats=True)
        nd = check_draws(got["draws"], g.w, p, q, budget, seed, ctx=f"p={p} q={q} budget={budget}")
        log(f"es p={p} q={q} budget={budget}: {nd} draws on a rounding boundary")
        mark = np.zeros(g.m, np.uint8)
        mark[got["draws"].astype(np.int64)] = 1
        assert got["stats"]["distinct_sampled"] == int(mark.sum())
        want = oracle.topk(g.n, g.src, g.dst, g.w, 100, p, edge_mark=mark)
        assert_parity(got, want, p, ei, ctx=f"es on the GPU's draws p={p} q={q}")
        if nd == 0:  # same draws: the oracle's own replay of the whole query agrees as well
            ref = oracle.sample_heavy_triangles(g.n, g.src, g.dst, g.w, 100, p, budget, seed, q=q)
            assert_parity(got, ref, p, ei, ctx=f"es replay p={p} q={q}")


def test_sampling_integer_exponent_draws_and_override(tt, small):
    """Integer q: the returned draws equal the oracle's draw for draw, with q named or implied,
    and the draws-only call (k = 0) returns the same sequence."""
    g, G = small
    ei = EdgeIndex(g.src, g.dst, g.w)
    for p, q in ((1.0, None), (2.0, None), (3.0, None), (-math.inf, 2.0), (0.0, 3.0), (1.5, 1.0)):
        got = G.sample(100, p, 50000, 21, q=q, return_draws=True)
        check_draws(got["draws"], g.w, p, q, 50000, 21, ctx=f"p={p} q={q}")
        want = oracle.sample_heavy_triangles(g.n, g.src, g.dst, g.w, 100, p, 50000, 21, q=q)
        assert_parity(got, want, p, ei, ctx=f"es p={p} q={q}")
        only = G.sample(0, p, 50000, 21, q=q, return_draws=True)
        assert only["n_out"] == 0 and np.array_equal(only["draws"], got["draws"])
    for bad in (0.0, -1.0, math.inf):
        with pytest.raises(tt.TopKError) as e:
            G.sample(10, 1.0, 100, 1, q=bad)
        assert e.value.code == tt.TT_E_ARG


@pytest.mark.parametrize("q", [2, 3])
def test_sampling_draw_target_above_2_64(tt, q):
    """Weights near 2^32 - 1 make Z = sum w^q exceed 2^64 (q = 2: ~m 2^64; q = 3: ~m 2^96), so the
    128-bit draw target x * floor(Z / 2^64) + floor(x * (Z mod 2^64) / 2^64) needs both terms.
    Draw for draw against the oracle, and the sampled top-k."""
    rng = np.random.default_rng(640 + q)
    n = 40
    s, d, _ = rand_graph(rng, n, 0.5)
    w = rng.integers(2**32 - 100000, 2**32, len(s), dtype=np.uint64).astype(np.uint32)
    w[rng.choice(len(w), size=len(w) // 3, replace=False)] = rng.integers(1, 1000, len(w) // 3).astype(np.uint32)
    assert sum(int(x) ** q for x in w.tolist()) >= 2**64
    ei = EdgeIndex(s, d, w)
    with tt.Graph(n, s, d, w) as G:
        for budget, seed in ((7, 1), (300, 2), (20000, 3)):
            got = G.sample(50, float(q), budget, seed, return_draws=True)
            check_draws(got["draws"], w, float(q), None, budget, seed, ctx=f"q={q} budget={budget}")
            want = oracle.sample_heavy_triangles(n, s, d, w, 50, float(q), budget, seed)
            assert_parity(got, want, float(q), ei, ctx=f"big-w es q={q} budget={budget}")


def test_sampling_converges_to_exact(tt, small):
    g, G = small
    exact = G.topk(100, 1.0)
    es = G.sample(100, 1.0, 50_000_000, 11)
    assert triples(es) == triples(exact) and np.array_equal(es["score"], exact["score"])
