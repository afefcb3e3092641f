"""CPU pins of the completeness certificate used on the graphs the oracle cannot enumerate
whole (tests/certificate.py): on graphs it can, the oracle's top-k of the certificate's
subgraph equals its top-k of the whole graph, for every form and every kind of p, and the
bounds hold for every triangle that scores at least S."""
import itertools
import math

import numpy as np
import pytest

import certificate
import graphgen
import oracle

ALL_P = [-math.inf, -3.0, -1.0, 0.0, 0.5, 1.0, 2.0, 3.0, math.inf]


@pytest.mark.parametrize("p", ALL_P)
def test_bounds_hold_for_every_triangle_above_s(p):
    g = graphgen.chung_lu(600, 6000, 2.3, 1.8, seed=31)
    i, j, l, w3 = oracle.list_triangles(g.n, g.src, g.dst, g.w)
    W = int(g.w.max())
    scores = np.array([oracle.score(p, int(a), int(b), int(c))[1] for a, b, c in w3])
    for S in np.quantile(scores, [0.5, 0.9, 0.99, 1.0]):
        a_min, y, z = certificate.bounds(p, float(S), W)
        srt = np.sort(w3, axis=1)[:, ::-1]
        above = scores >= S
        assert np.all(srt[above, 0] >= a_min) and np.all(srt[above, 1] >= y) and np.all(srt[above, 2] >= z)


@pytest.mark.parametrize("p", ALL_P)
@pytest.mark.parametrize("k", [1, 50, 600])
def test_subgraph_top_k_is_the_top_k(p, k, monkeypatch):
    g = graphgen.chung_lu(3000, 40000, 2.2, 1.8, seed=32, plant=6, plant_size=4, plant_mult=1000)
    want = oracle.topk(g.n, g.src, g.dst, g.w, k, p)
    S = float(want["score"][-1])
    monkeypatch.setattr(certificate, "CHUNK", 4096)  # several chunks
    sizes = {}
    for form in ("all-edges", "two-edge", "one-edge", None):
        sel, desc = certificate.subgraph(g.n, g.src, g.dst, g.w, p, S, form=form)
        sizes[desc["form"]] = len(sel)
        got = oracle.topk(g.n, g.src[sel], g.dst[sel], g.w[sel], k, p)
        for x in ("i", "j", "l", "score"):
            assert np.array_equal(got[x], want[x]), (desc, x)
    # the vertex-restricted answer is kept as well (served subset requests)
    vm = np.zeros(g.n, np.uint8)
    vm[np.arange(0, g.n, 7)] = 1
    want = oracle.topk(g.n, g.src, g.dst, g.w, k, p, vertex_mark=vm)
    if want["n_out"]:
        sel, desc = certificate.subgraph(g.n, g.src, g.dst, g.w, p, float(want["score"][-1]), form="two-edge")
        got = oracle.topk(g.n, g.src[sel], g.dst[sel], g.w[sel], k, p, vertex_mark=vm)
        assert got["i"].tolist() == want["i"].tolist() and got["l"].tolist() == want["l"].tolist()


def test_wedge_pairs_brute_force():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 30, 80)
    b = (a + rng.integers(1, 29, 80)) % 30
    keys = set(certificate.pair_keys(a, b).tolist())
    a, b = np.array([k >> 32 for k in keys]), np.array([k & 0xFFFFFFFF for k in keys])
    got = set(certificate._wedge_pairs(a, b).tolist())
    nb = {v: set() for v in range(30)}
    for x, y in zip(a.tolist(), b.tolist()):
        nb[x].add(y)
        nb[y].add(x)
    want = set()
    for v in range(30):
        for x, y in itertools.combinations(sorted(nb[v]), 2):
            want.add((min(x, y) << 32) | max(x, y))
    assert got == want


@pytest.mark.parametrize("p", ALL_P)
@pytest.mark.parametrize("k", [1, 40, 700])
def test_certified_topk_is_the_top_k(p, k, monkeypatch):
    """certified_topk (lower bound from k real triangles, then the certified subgraph) returns
    the oracle's whole-graph answer, also restricted to a vertex subset."""
    g = graphgen.chung_lu(4000, 50000, 2.2, 1.8, seed=33, plant=5, plant_size=4, plant_mult=1000)
    monkeypatch.setattr(certificate, "CHUNK", 8192)
    for vm in (None, (np.arange(g.n) % 5 == 0).astype(np.uint8)):
        want = oracle.topk(g.n, g.src, g.dst, g.w, k, p, vertex_mark=vm)
        got, desc = certificate.certified_topk(g.n, g.src, g.dst, g.w, k, p, vertex_mark=vm)
        for x in ("i", "j", "l", "score"):
            assert np.array_equal(got[x], want[x]), (p, k, desc, x)


def test_triangles_from_marked_edges_brute_force():
    """The oracle's enumeration from the marked edges finds exactly the triangles with a marked
    edge, each once (brute force over all triples)."""
    import brute
    rng = np.random.default_rng(44)
    for trial in range(6):
        n = int(rng.integers(6, 30))
        iu = np.array(list(itertools.combinations(range(n), 2)), np.uint32)
        e = iu[rng.random(len(iu)) < 0.5]
        s, d = e[:, 0].copy(), e[:, 1].copy()
        w = rng.integers(1, 9, len(s)).astype(np.uint32)
        em = (rng.random(len(s)) < 0.3).astype(np.uint8)
        marked = {(int(a), int(b)) for a, b, x in zip(s, d, em) if x}
        tris = [t for t in brute.all_triangles(n, s, d, w)
                if (t[0], t[1]) in marked or (t[0], t[2]) in marked or (t[1], t[2]) in marked]
        tris.sort(key=lambda t: (-(t[3] + t[4] + t[5]), t[0], t[1], t[2]))
        out = oracle.topk(n, s, d, w, 10**6, 1.0, edge_mark=em, from_marked_edges=True)
        assert out["total"] == len(tris)
        assert list(zip(out["i"].tolist(), out["j"].tolist(), out["l"].tolist())) == [t[:3] for t in tris]
