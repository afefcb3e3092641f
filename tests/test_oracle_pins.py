"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Every test here runs on the CPU.  Each one is chosen so that a plausible mistake in the
oracle (a dropped term, a wrong sign or index, a swapped weight, an off-by-one in the
sampler's CDF) fails it:

* closed-form means (Eq. 1 and the special cases named after it), in tests/golden/scores.txt
* invariants of the p-mean: constant triples, homogeneity, the power-mean inequality, limits
* enumeration: brute force over all triples, C(n,3) for K_n, trace(A^3)/6, trees, bipartite
  graphs and wheels
* selection: uniform weights (pure tie-break), planted dominant cliques, K_n with w_ij=i+j+2
* weighted edge sampling (Alg. 3): the published SplitMix64 sequence, Prop. 1 frequencies,
  the union semantics against a brute-force replay, and convergence to the exact top-k.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import brute
import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALL_P = [-math.inf, -3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 1.5, 2.0, 3.0, math.inf]


def _pval(s):
    return {"inf": math.inf, "-inf": -math.inf}.get(s, None) if s in ("inf", "-inf") else float(s)


def _rand_graph(rng, n, prob, wlo=1, whi=20):
    src, dst = [], []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < prob:
                if rng.random() < 0.5:
                    src.append(i); dst.append(j)
                else:
                    src.append(j); dst.append(i)
    w = rng.integers(wlo, whi + 1, len(src))
    return np.array(src, np.uint32), np.array(dst, np.uint32), np.array(w, np.uint32)


# ---------------------------------------------------------------------------------- scoring

def test_golden_closed_forms():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "scores.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 10
    for p, a, b, c, v in rows:
        _, s = oracle.score(_pval(p), int(a), int(b), int(c))
        assert s == pytest.approx(float(v), rel=1e-15, abs=0), (p, a, b, c, s, v)


def test_exact_keys_closed_forms():
    assert oracle.score(1, 1, 2, 3)[0] == 6
    assert oracle.score(2, 1, 5, 7)[0] == 75
    assert oracle.score(0, 1, 2, 4)[0] == 8
    assert oracle.score(math.inf, 1, 2, 9)[0] == 9
    assert oracle.score(-math.inf, 1, 2, 9)[0] == 1
    # widest keys: product of three 2^32-1 needs 96 bits, sum of squares 66 bits
    big = 2**32 - 1
    assert oracle.score(0, big, big, big)[0] == big**3
    assert oracle.score(2, big, big, big)[0] == 3 * big * big


@pytest.mark.parametrize("p", ALL_P)
def test_constant_triple_is_its_own_mean(p):
    for c in (1, 2, 7, 1000, 123456, 2**32 - 1):
        assert oracle.score(p, c, c, c)[1] == pytest.approx(c, rel=1e-15)


@pytest.mark.parametrize("p", [-3.0, -1.0, -0.5, 0.5, 1.5, 3.0])
def test_homogeneity(p):
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b, c = (int(x) for x in rng.integers(1, 10**4, 3))
        lam = int(rng.integers(2, 50))
        s1 = oracle.score(p, a, b, c)[1]
        s2 = oracle.score(p, lam * a, lam * b, lam * c)[1]
        assert s2 == pytest.approx(lam * s1, rel=2e-15)


def test_power_mean_inequality_and_bounds():
    """m_p is non-decreasing in p and lies between min and max; p=-1 is the harmonic mean."""
    rng = np.random.default_rng(2)
    ps = [-math.inf, -50.0, -3.0, -1.0, -0.5, -1e-6, 0.0, 1e-6, 0.5, 1.0, 2.0, 3.0, 50.0, math.inf]
    for _ in range(300):
        a, b, c = (int(x) for x in rng.integers(1, 10**6, 3))
        vals = [oracle.score(p, a, b, c)[1] for p in ps]
        for x, y in zip(vals, vals[1:]):
            assert y >= x * (1 - 1e-15)
        assert vals[0] == min(a, b, c) and vals[-1] == max(a, b, c)
        harm = 3.0 / (1.0 / a + 1.0 / b + 1.0 / c)
        assert oracle.score(-1.0, a, b, c)[1] == pytest.approx(harm, rel=1e-14)
        ari = (a + b + c) / 3.0
        assert oracle.score(1.0, a, b, c)[1] == ari
        assert oracle.score(2.0, a, b, c)[1] == pytest.approx(math.sqrt((a * a + b * b + c * c) / 3.0), rel=1e-15)


def test_limits():
    """p -> 0 tends to the geometric mean; p -> +-inf to max / min (Sec. 1's special cases)."""
    rng = np.random.default_rng(3)
    for _ in range(100):
        a, b, c = (int(x) for x in rng.integers(1, 10**6, 3))
        geo = (a * b * c) ** (1.0 / 3.0)
        for p in (1e-9, -1e-9):
            assert oracle.score(p, a, b, c)[1] == pytest.approx(geo, rel=1e-8)
        mx, mn = max(a, b, c), min(a, b, c)
        for p in (200.0, 1000.0):
            s = oracle.score(p, a, b, c)[1]
            assert mx * 3 ** (-1.0 / p) * (1 - 1e-15) <= s <= mx
            s = oracle.score(-p, a, b, c)[1]
            assert mn <= s <= mn * 3 ** (1.0 / p) * (1 + 1e-15)


@pytest.mark.parametrize("p", [-math.inf, 0.0, 1.0, 2.0, math.inf])
def test_exact_key_orders_like_the_score(p):
    rng = np.random.default_rng(4)
    trip = [tuple(int(x) for x in rng.integers(1, 60, 3)) for _ in range(400)]
    ks = [oracle.score(p, *t) for t in trip]
    for (k1, s1), (k2, s2) in itertools.combinations(ks[:120], 2):
        if k1 > k2:
            assert s1 >= s2
        if k1 == k2:
            assert s1 == s2


def test_generic_key_is_the_double_score():
    for p in (-1.0, 0.5, 1.5, 3.0):
        k, s = oracle.score(p, 3, 8, 20)
        assert np.array([s]).view(np.uint64)[0] == k


# ---------------------------------------------------------------------------------- validation

def test_validation_codes():
    ok = ([0, 1, 2], [1, 2, 0], [1, 1, 1])
    assert oracle.validate(3, *ok) == oracle.OK
    assert oracle.validate(3, [0, 1], [1, 1], [1, 1]) == oracle.E_SELF_LOOP
    assert oracle.validate(3, [0, 1], [1, 0], [1, 1]) == oracle.E_DUP_EDGE
    assert oracle.validate(3, [0, 1], [1, 2], [1, 0]) == oracle.E_ZERO_WEIGHT
    assert oracle.validate(3, [0, 1], [1, 3], [1, 1]) == oracle.E_VERTEX_RANGE
    assert oracle.validate(0, [], [], []) == oracle.OK
    with pytest.raises(oracle.OracleError) as e:
        oracle.topk(3, [0, 0], [1, 1], [1, 1], 5, 1.0)
    assert e.value.code == oracle.E_DUP_EDGE


# Several faults in one input: the first failing rule in the order vertex range, self-loop,
# zero weight, duplicate pair is reported (the reading of the simple-graph, positive-weight
# requirement of Sec. 1), whatever the order of the faulty edges in the list.
MULTI_FAULT = [
    # (n, src, dst, w, expected)
    (4, [0, 1, 2, 3], [1, 1, 3, 5], [1, 1, 1, 1], oracle.E_VERTEX_RANGE),        # loop, then range
    (4, [0, 3, 1], [7, 3, 2], [0, 1, 1], oracle.E_VERTEX_RANGE),                 # range+zero, loop
    (4, [0, 2, 1, 0], [1, 2, 0, 3], [1, 1, 1, 0], oracle.E_SELF_LOOP),           # loop, dup, zero
    (4, [1, 0, 3], [0, 1, 3], [0, 1, 1], oracle.E_SELF_LOOP),                    # zero+dup, loop
    (4, [0, 1, 2, 1], [1, 0, 3, 2], [1, 1, 0, 1], oracle.E_ZERO_WEIGHT),         # dup before zero
    (4, [0, 1, 2, 3, 3], [1, 2, 0, 0, 2], [1, 1, 1, 1, 0], oracle.E_ZERO_WEIGHT),
    (5, [0, 1, 0, 2, 4, 3], [1, 0, 2, 0, 3, 4], [1, 1, 1, 1, 1, 1], oracle.E_DUP_EDGE),  # three repeats
]


@pytest.mark.parametrize("case", range(len(MULTI_FAULT)))
def test_validation_precedence_with_several_faults(case):
    n, s, d, w, want = MULTI_FAULT[case]
    assert oracle.validate(n, s, d, w) == want
    # the same edges in reverse order report the same rule
    assert oracle.validate(n, s[::-1], d[::-1], w[::-1]) == want


# ---------------------------------------------------------------------------------- enumeration

@pytest.mark.parametrize("seed", range(6))
def test_listing_matches_all_triples(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 28))
    s, d, w = _rand_graph(rng, n, rng.uniform(0.15, 0.7))
    want = sorted(brute.all_triangles(n, s, d, w))
    i, j, l, w3 = oracle.list_triangles(n, s, d, w)
    got = sorted((int(a), int(b), int(c), int(x), int(y), int(z)) for a, b, c, (x, y, z) in zip(i, j, l, w3))
    assert got == want


@pytest.mark.parametrize("nn", [3, 4, 50, 200])
def test_complete_graph_count(nn):
    s, d = zip(*itertools.combinations(range(nn), 2))
    w = np.ones(len(s), np.uint32)
    assert oracle.count_triangles(nn, s, d, w) == math.comb(nn, 3)


def test_trace_a3_over_6(small_graph):
    g = small_graph
    A = np.zeros((g.n, g.n), np.float64)
    A[g.src, g.dst] = 1
    A[g.dst, g.src] = 1
    t6 = np.trace(A @ A @ A)  # exact: every entry of A^2 is below 2^53
    assert t6 % 6 == 0
    assert oracle.count_triangles(g.n, g.src, g.dst, g.w) == int(t6) // 6


def test_trees_and_bipartite_have_no_triangles():
    rng = np.random.default_rng(5)
    n = 500
    parent = [int(rng.integers(0, v)) for v in range(1, n)]
    s = np.array(parent, np.uint32)
    d = np.arange(1, n, dtype=np.uint32)
    assert oracle.count_triangles(n, s, d, np.ones(n - 1, np.uint32)) == 0
    a, b = 30, 40
    s, d = zip(*[(x, a + y) for x in range(a) for y in range(b)])
    assert oracle.count_triangles(a + b, s, d, np.ones(len(s), np.uint32)) == 0


@pytest.mark.parametrize("r", [4, 5, 17])
def test_wheel(r):
    # hub 0, rim 1..r in a cycle: exactly the r triangles (0, t, t+1)
    s = [0] * r + list(range(1, r + 1))
    d = list(range(1, r + 1)) + [t % r + 1 for t in range(1, r + 1)]
    w = [1] * (2 * r)
    out = oracle.topk(r + 1, s, d, w, 100, 1.0)
    assert out["total"] == r
    got = sorted(zip(out["i"].tolist(), out["j"].tolist(), out["l"].tolist()))
    want = sorted([(0, t, t + 1) for t in range(1, r)] + [(0, 1, r)])
    assert got == want


# ---------------------------------------------------------------------------------- selection

@pytest.mark.parametrize("p", ALL_P)
@pytest.mark.parametrize("seed", range(3))
def test_topk_matches_brute_force(p, seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(8, 26))
    s, d, w = _rand_graph(rng, n, 0.5, 1, 6)  # narrow weights: many ties
    k = int(rng.integers(1, 40))
    want, total = brute.topk(n, s, d, w, k, p)
    out = oracle.topk(n, s, d, w, k, p)
    assert out["total"] == total
    assert out["n_out"] == min(k, total)
    got = list(zip(out["i"].tolist(), out["j"].tolist(), out["l"].tolist()))
    if p in oracle.EXACT_P:
        assert got == [t[:3] for t in want]
    else:
        # generic p: scores agree to 1e-12; any set difference lies at the k-th score
        ws = [brute.float_mean(p, *t[3:]) for t in want]
        for sc, ref in zip(out["score"], ws):
            assert sc == pytest.approx(ref, rel=1e-12)
        if want:
            kth = ws[-1]
            diff = set(got) ^ {t[:3] for t in want}
            allt = {t[:3]: brute.float_mean(p, *t[3:]) for t in brute.all_triangles(n, s, d, w)}
            for t in diff:
                assert allt[t] == pytest.approx(kth, rel=1e-12)


def test_uniform_weights_give_lexicographic_order():
    rng = np.random.default_rng(6)
    n = 40
    s, d, _ = _rand_graph(rng, n, 0.35)
    w = np.full(len(s), 7, np.uint32)
    tris = sorted(t[:3] for t in brute.all_triangles(n, s, d, w))
    for p in (-math.inf, -1.0, 0.0, 1.0, 2.5, math.inf):
        out = oracle.topk(n, s, d, w, 25, p)
        assert list(zip(out["i"].tolist(), out["j"].tolist(), out["l"].tolist())) == tris[:25]
        assert np.allclose(out["score"], 7.0, rtol=1e-15)


@pytest.mark.parametrize("p", [-math.inf, -1.0, 0.0, 1.0, 2.0, math.inf])
def test_planted_dominant_cliques(p):
    """Planted 4-cliques whose weights exceed every natural weight hold the top 4c triangles.

    The cliques sit on fresh vertices; each planted vertex also gets light edges to its own
    natural vertices (no two planted vertices share one), so the only triangles that contain
    a planted edge are the 4c planted ones, and every other triangle is strictly lighter."""
    g = graphgen.chung_lu(3000, 30000, 2.3, 1.8, seed=11)
    rng = np.random.default_rng(7)
    c = 5
    members = (g.n + rng.permutation(4 * c)).reshape(c, 4)
    E = {(min(a, b), max(a, b)): x for a, b, x in zip(g.src.tolist(), g.dst.tolist(), g.w.tolist())}
    attach = rng.choice(g.n, size=(4 * c, 3), replace=False)
    for v, nat in zip(members.reshape(-1).tolist(), attach):
        for x in nat.tolist():
            E[(x, v)] = int(rng.integers(1, 100))
    for q in range(c):
        for a, b in itertools.combinations(sorted(members[q].tolist()), 2):
            E[(a, b)] = int(rng.integers(10**9, 2 * 10**9))
    s, d = zip(*E.keys())
    w = list(E.values())
    planted = []
    for q in range(c):
        for a, b, l in itertools.combinations(sorted(members[q].tolist()), 3):
            x, y, z = E[(a, b)], E[(a, l)], E[(b, l)]
            val = brute.exact_rank_value(p, x, y, z) if p in oracle.EXACT_P else brute.float_mean(p, x, y, z)
            planted.append((-val, a, b, l))
    planted.sort()
    out = oracle.topk(g.n + 4 * c, s, d, w, 4 * c + 1, p)
    got = list(zip(out["i"].tolist(), out["j"].tolist(), out["l"].tolist()))
    assert got[:4 * c] == [t[1:] for t in planted]
    assert out["score"][4 * c] <= 10**6  # the next one is a natural triangle


def test_complete_graph_with_additive_weights():
    """K_n with w_ij = (i+1) + (j+1): m_1 = 2(i+j+l+3)/3, so the top-k is the triples with the
    largest i+j+l, ties in lexicographic order."""
    n = 30
    s, d = zip(*itertools.combinations(range(n), 2))
    w = [a + b + 2 for a, b in zip(s, d)]
    out = oracle.topk(n, s, d, w, 200, 1.0)
    want = sorted(itertools.combinations(range(n), 3), key=lambda t: (-sum(t), t))[:200]
    assert list(zip(out["i"].tolist(), out["j"].tolist(), out["l"].tolist())) == want
    assert out["score"][0] == 2.0 * (n - 1)
    for (i, j, l), sc in zip(want, out["score"]):
        assert sc == 2.0 * (i + j + l + 3) / 3.0


def test_fewer_than_k_and_k_zero():
    s, d, w = [0, 1, 2, 2], [1, 2, 0, 3], [5, 6, 7, 1]
    out = oracle.topk(4, s, d, w, 10, 1.0)
    assert out["n_out"] == 1 and out["total"] == 1
    assert (out["i"][0], out["j"][0], out["l"][0]) == (0, 1, 2)
    assert out["score"][0] == 6.0
    assert oracle.topk(4, s, d, w, 0, 1.0)["n_out"] == 0
    assert oracle.topk(5, [], [], [], 3, 1.0)["n_out"] == 0


def test_edge_and_vertex_filters_together():
    """Both marks: a triangle is admitted when it has a marked edge AND a marked vertex."""
    rng = np.random.default_rng(18)
    n = 26
    s, d, w = _rand_graph(rng, n, 0.5, 1, 12)
    vm = np.zeros(n, np.uint8)
    vm[[2, 9, 17]] = 1
    em = (rng.random(len(s)) < 0.3).astype(np.uint8)
    E = brute.edge_dict(s, d, w)
    marked = {(min(int(a), int(b)), max(int(a), int(b))) for a, b, x in zip(s, d, em) if x}
    tris = [t for t in brute.all_triangles(n, s, d, w)
            if (vm[t[0]] or vm[t[1]] or vm[t[2]])
            and ((t[0], t[1]) in marked or (t[0], t[2]) in marked or (t[1], t[2]) in marked)]
    tris.sort(key=lambda t: (-(t[3] + t[4] + t[5]), t[0], t[1], t[2]))
    out = oracle.topk(n, s, d, w, 12, 1.0, edge_mark=em, vertex_mark=vm)
    assert out["total"] == len(tris) and len(E) == len(s)
    assert list(zip(out["i"].tolist(), out["j"].tolist(), out["l"].tolist())) == [t[:3] for t in tris[:12]]
    only_e = oracle.topk(n, s, d, w, 0, 1.0, edge_mark=em)["total"]
    only_v = oracle.topk(n, s, d, w, 0, 1.0, vertex_mark=vm)["total"]
    assert len(tris) <= min(only_e, only_v)


def test_vertex_filter_matches_brute_force():
    rng = np.random.default_rng(8)
    n = 24
    s, d, w = _rand_graph(rng, n, 0.45, 1, 9)
    mark = np.zeros(n, np.uint8)
    mark[[3, 11]] = 1
    tris = [t for t in brute.all_triangles(n, s, d, w) if mark[t[0]] or mark[t[1]] or mark[t[2]]]
    tris.sort(key=lambda t: (-(t[3] + t[4] + t[5]), t[0], t[1], t[2]))
    out = oracle.topk(n, s, d, w, 15, 1.0, vertex_mark=mark)
    assert out["total"] == len(tris)
    assert list(zip(out["i"].tolist(), out["j"].tolist(), out["l"].tolist())) == [t[:3] for t in tris[:15]]


# ---------------------------------------------------------------------------------- sampling

def test_splitmix64_reference_sequence():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.strip() and not l.startswith("#")]
    for idx, val in rows:
        assert oracle.splitmix64(1234567, int(idx)) == int(val)


def test_sample_exponent_reading():
    assert oracle.sample_exponent(1.0) == 1.0
    assert oracle.sample_exponent(2.0) == 2.0
    assert oracle.sample_exponent(0.5) == 0.5
    for p in (0.0, -1.0, -math.inf, math.inf):
        assert oracle.sample_exponent(p) == 1.0


@pytest.mark.parametrize("p", [1.0, 2.0, 3.0, 0.5, 1.5])
def test_prop1_edge_frequencies(p):
    """Each draw picks edge e with probability w_e^q / Z (Alg. 3), so a triangle is hit in a
    draw with probability w_q(t) / Z (Prop. 1).  Binomial 5-sigma bands over 4e5 draws."""
    w = np.array([1, 2, 3, 5, 8, 1, 4, 7, 2], np.uint32)
    T = 400_000
    _, draws = oracle.es_draw(w, p, T, seed=12345, return_draws=True)
    q = oracle.sample_exponent(p)
    prob = w.astype(np.float64) ** q
    prob /= prob.sum()
    cnt = np.bincount(draws.astype(np.int64), minlength=len(w))
    for e in range(len(w)):
        sd = math.sqrt(T * prob[e] * (1 - prob[e]))
        assert abs(cnt[e] - T * prob[e]) <= 5 * sd + 1, (e, cnt[e], T * prob[e])
    # Prop. 1 for the triangle on edges 0, 1, 2 (their draws are disjoint events)
    hit = np.isin(draws, [0, 1, 2]).sum()
    pt = prob[:3].sum()
    assert abs(hit - T * pt) <= 5 * math.sqrt(T * pt * (1 - pt))


def test_exact_draw_is_inverse_cdf():
    """Integer q: draw s selects the first edge whose inclusive prefix exceeds
    floor(x_s * Z / 2^64), x_s the s-th SplitMix64 output (a from-scratch replay)."""
    w = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.uint32)
    for q in (1, 2, 3):
        pref = np.cumsum([int(x) ** q for x in w.tolist()])
        Z = int(pref[-1])
        _, draws = oracle.es_draw(w, float(q), 300, seed=99, return_draws=True)
        for s in range(300):
            r = (oracle.splitmix64(99, s) * Z) >> 64
            want = next(e for e in range(len(w)) if int(pref[e]) > r)
            assert int(draws[s]) == want


def _replay_exact(w, q, seed, budget):
    """The integer-q draw rule in Python integers: r = floor(x Z / 2^64), first e with
    prefix[e] > r (bisect), for the first `budget` SplitMix64 outputs."""
    import bisect
    pref = list(itertools.accumulate(int(x) ** q for x in w.tolist()))
    Z = pref[-1]
    return Z, [bisect.bisect_right(pref, (oracle.splitmix64(seed, s) * Z) >> 64) for s in range(budget)]


@pytest.mark.parametrize("case", ["near_2_32_q2", "near_2_32_q3", "planted_x1000_q3"])
def test_exact_draw_target_above_2_64(case):
    """Integer q with Z >= 2^64: the draw target floor(x Z / 2^64) has a high part x * floor(Z /
    2^64) as well as the carry of x * (Z mod 2^64); dropping either term moves the draws.  Weights
    near 2^32 - 1 at q = 2 and 3, and Zipf(1.8) weights with a few planted x1000 edges (the
    1M-vertex workload's weight recipe) at q = 3."""
    rng = np.random.default_rng(64)
    if case.startswith("near_2_32"):
        w = rng.integers(2**32 - 5000, 2**32, 257, dtype=np.uint64).astype(np.uint32)
        q = 2 if case.endswith("q2") else 3
    else:
        w = graphgen.zipf(4_000_000, 1.8, seed=7)  # its w^3 tail alone reaches Z > 2^64
        hot = rng.choice(len(w), size=300, replace=False)
        w[hot] = (w[hot].astype(np.uint64) * 1000).astype(np.uint32)
        q = 3
    budget, seed = 4000, 2024 + q
    Z, want = _replay_exact(w, q, seed, budget)
    assert Z >= 2**64, Z
    _, draws = oracle.es_draw(w, float(q), budget, seed=seed, return_draws=True)
    assert draws.astype(np.int64).tolist() == want
    # the high term matters: a target without x * floor(Z / 2^64) picks other edges
    pref = list(itertools.accumulate(int(x) ** q for x in w.tolist()))
    import bisect
    lo_only = [bisect.bisect_right(pref, (oracle.splitmix64(seed, s) * (Z % 2**64)) >> 64) for s in range(50)]
    assert lo_only != want[:50]


def test_draw_with_q_override():
    """The sampling exponent can be named (Alg. 3 samples by w^q; q = p is the default reading
    for finite p > 0): the draws with q given equal the draws of p = q, for any p, and a
    non-integer q draws the first edge whose FP64 prefix of w^q exceeds (x >> 11) 2^-53 Z."""
    w = graphgen.zipf(5000, 1.8, seed=3)
    for q in (1.0, 2.0, 0.5, 1.5):
        a = oracle.es_draw(w, q, 3000, 77, return_draws=True)[1]
        for p in (q, -1.0, math.inf, 0.0):
            b = oracle.es_draw(w, p, 3000, 77, return_draws=True, q=q)[1]
            assert np.array_equal(a, b), (q, p)
    for q in (0.5, 1.5, 2.5):
        P = oracle.es_prefix_f64(w, q)
        # the prefix is the running sum of w^q: its total agrees with an exactly rounded sum
        assert abs(P[-1] - math.fsum(float(x) ** q for x in w.tolist())) <= 1e-12 * P[-1]
        assert np.all(np.diff(P) > 0)
        _, draws = oracle.es_draw(w, 1.0, 2000, 5, return_draws=True, q=q)
        for s in range(2000):
            r = float(oracle.splitmix64(5, s) >> 11) * 2.0**-53 * P[-1]
            e = int(draws[s])
            assert P[e] > r and (e == 0 or P[e - 1] <= r), (q, s)
    with pytest.raises(oracle.OracleError):
        oracle.es_draw(w, 1.0, 10, 1, q=0.0)
    with pytest.raises(oracle.OracleError):
        oracle.es_draw(w, 1.0, 10, 1, q=math.inf)


@pytest.mark.parametrize("seed", range(3))
def test_es_union_matches_replay(seed):
    rng = np.random.default_rng(300 + seed)
    n = 22
    s, d, w = _rand_graph(rng, n, 0.45, 1, 30)
    budget = 12
    mark, draws = oracle.es_draw(w, 1.0, budget, seed=seed, return_draws=True)
    E = brute.edge_dict(s, d, w)
    adj = {v: set() for v in range(n)}
    for a, b in E:
        adj[a].add(b); adj[b].add(a)
    T = set()
    for e in draws.tolist():
        a, b = int(s[e]), int(d[e])
        for c in adj[a] & adj[b]:
            T.add(tuple(sorted((a, b, c))))
    ranked = sorted(T, key=lambda t: (-(E[(t[0], t[1])] + E[(t[0], t[2])] + E[(t[1], t[2])]), t))
    out = oracle.sample_heavy_triangles(n, s, d, w, 10, 1.0, budget, seed)
    assert out["total"] == len(T)
    assert list(zip(out["i"].tolist(), out["j"].tolist(), out["l"].tolist())) == ranked[:10]


def test_es_with_large_budget_is_exact():
    """With s >= log(1/delta)/q draws every edge is found w.p. >= 1-delta (Sec. 4.4)."""
    g = graphgen.chung_lu(300, 1500, 2.5, 2.0, seed=5)
    q_min = float(g.w.min()) / float(g.w.sum())
    budget = int(math.log(1e9 * g.m) / q_min) + 1
    exact = oracle.topk(g.n, g.src, g.dst, g.w, 50, 1.0)
    es = oracle.sample_heavy_triangles(g.n, g.src, g.dst, g.w, 50, 1.0, budget, seed=3)
    assert es["distinct_edges"] == g.m
    for x in ("i", "j", "l", "score"):
        assert es[x].tolist() == exact[x].tolist(), x


# ---------------------------------------------------------------------------------- cliques (Sec. 4.5)

def _brute_cliques(n, s, d, w, size, p):
    E = brute.edge_dict(s, d, w)
    out = []
    for vs in itertools.combinations(range(n), size):
        ws = [E.get(pair) for pair in itertools.combinations(vs, 2)]
        if all(x is not None for x in ws):
            out.append((vs, ws))
    return out


@pytest.mark.parametrize("size", [4, 5])
@pytest.mark.parametrize("p", [1.0, math.inf, -math.inf, 0.5, 0.0, 2.0])
def test_cliques_match_all_subsets(size, p):
    """Every clique of the given size, found by brute force over all vertex subsets, ranked by
    the p-mean of its edges (exact rationals at p = 1, max/min at +-inf, the float formula of
    Eq. 1 elsewhere), ties by the sorted IDs."""
    rng = np.random.default_rng(70 + size)
    n = 14
    s, d, w = _rand_graph(rng, n, 0.7, 1, 9)
    cl = _brute_cliques(n, s, d, w, size, p)
    E = size * (size - 1) // 2
    if p == 1.0:
        val = lambda ws: Fraction(sum(ws), E)  # noqa: E731
    elif math.isinf(p):
        val = (lambda ws: max(ws)) if p > 0 else (lambda ws: min(ws))  # noqa: E731
    elif p == 0.0:
        val = lambda ws: math.exp(sum(math.log(x) for x in ws) / E)  # noqa: E731
    else:
        val = lambda ws: (sum(x ** p for x in ws) / E) ** (1.0 / p)  # noqa: E731
    cl.sort(key=lambda c: (-val(c[1]), c[0]))
    out = oracle.cliques(n, s, d, w, size, 10**6, p)
    assert out["total"] == len(cl)
    got = [tuple(v) for v in out["v"].tolist()]
    if p in (1.0, math.inf, -math.inf):
        assert got == [c[0] for c in cl]
        assert all(float(val(c[1])) == sc for c, sc in zip(cl, out["score"]))
    else:
        ref = np.array([val(c[1]) for c in cl])
        assert np.allclose(np.sort(out["score"])[::-1], np.sort(ref)[::-1], rtol=1e-12, atol=0)


@pytest.mark.parametrize("nn,size", [(8, 4), (9, 5), (12, 4)])
def test_complete_graph_clique_counts(nn, size):
    s, d = (np.array(x, np.uint32) for x in zip(*itertools.combinations(range(nn), 2)))
    out = oracle.cliques(nn, s, d, np.full(len(s), 3, np.uint32), size, 5, 1.0)
    assert out["total"] == math.comb(nn, size)
    # uniform weights: the lexicographically first subsets
    assert [tuple(v) for v in out["v"].tolist()] == list(itertools.islice(itertools.combinations(range(nn), size), 5))


def test_cliques_on_marked_edges():
    rng = np.random.default_rng(75)
    n = 16
    s, d, w = _rand_graph(rng, n, 0.6, 1, 20)
    em = (rng.random(len(s)) < 0.2).astype(np.uint8)
    marked = {(min(int(a), int(b)), max(int(a), int(b))) for a, b, x in zip(s, d, em) if x}
    cl = [c for c in _brute_cliques(n, s, d, w, 4, 1.0) if any(pr in marked for pr in itertools.combinations(c[0], 2))]
    cl.sort(key=lambda c: (-sum(c[1]), c[0]))
    out = oracle.cliques(n, s, d, w, 4, 10**6, 1.0, edge_mark=em)
    assert out["total"] == len(cl) and [tuple(v) for v in out["v"].tolist()] == [c[0] for c in cl]
