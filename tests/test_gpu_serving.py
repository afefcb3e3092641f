"""Served form: a continuous-batching request loop over one resident graph.

Every request's result must equal the single-query result for the same arguments (alone vs in
the mix), admission must respect the scratch budget, and results are checked against the
oracle for a sample of requests."""
import ctypes
import math
import sys

import numpy as np
import pytest

import graphgen
import oracle
from paritylib import EdgeIndex, assert_parity, triples

pytestmark = pytest.mark.gpu

P_CHOICES = (-math.inf, -1.0, 0.0, 1.0, 2.0, math.inf)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def tt():
    import paper_1910_00692_amd as tt
    tt.library()
    return tt


@pytest.fixture(scope="module")
def graph(tt):
    g = graphgen.chung_lu(100_000, 1_000_000, 2.1, 1.8, seed=4)
    G = tt.Graph(g.n, g.src, g.dst, g.w)
    yield g, G
    G.close()


def requests(n, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(np.floor(np.exp(rng.uniform(math.log(10), math.log(10_000)))))
        p = float(P_CHOICES[rng.integers(0, len(P_CHOICES))])
        sub = None
        if rng.random() < 0.2:
            sub = np.sort(rng.choice(n, size=1000, replace=False)).astype(np.uint32)
        out.append((k, p, sub))
    return out


def same(a, b):
    return a["n_out"] == b["n_out"] and triples(a) == triples(b) and np.array_equal(a["score"], b["score"])


def test_served_equals_single(tt, graph):
    g, G = graph
    reqs = requests(g.n, 48, 7)
    singles = [G.topk(k, p, subset=sub) for k, p, sub in reqs]
    log("singles done")
    with tt.Server(G, slots=4, scratch_budget=8 << 30) as S:
        tickets = [S.submit(k, p, sub) for k, p, sub in reqs]
        served = [S.wait(t) for t in tickets]
        info = S.info()
    log(f"server info {info}")
    for (k, p, sub), a, b in zip(reqs, singles, served):
        assert same(a, b), (k, p, sub is not None)
    assert info["completed"] == len(reqs) and info["admitted"] == len(reqs)
    assert info["max_running"] >= 2  # requests overlapped on the device


def test_served_with_stream_placed_in_parts(tt, graph, monkeypatch):
    """A fresh graph whose weight-ordered stream is placed bin range by bin range (as on graphs
    of more than 2^27 entries), first needed by requests running concurrently: each served
    result equals the single-query result of the graph that placed the stream at once."""
    g, G = graph
    reqs = [r for r in requests(g.n, 64, 19) if r[2] is None][:32]
    singles = [G.topk(k, p) for k, p, _ in reqs]
    monkeypatch.setenv("TT_WS_ALL_AT_ONCE", "0")
    with tt.Graph(g.n, g.src, g.dst, g.w) as H:
        with tt.Server(H, slots=4, scratch_budget=8 << 30) as S:
            tickets = [S.submit(k, p, None) for k, p, _ in reqs]
            served = [S.wait(t) for t in tickets]
            info = S.info()
    log(f"server info {info}")
    for (k, p, _), a, b in zip(reqs, singles, served):
        assert same(a, b), (k, p)
    assert info["max_running"] >= 2


def test_served_against_oracle(tt, graph):
    g, G = graph
    ei = EdgeIndex(g.src, g.dst, g.w)
    reqs = requests(g.n, 6, 11)
    with tt.Server(G, slots=3, scratch_budget=8 << 30) as S:
        tickets = [S.submit(k, p, sub) for k, p, sub in reqs]
        for (k, p, sub), t in zip(reqs, tickets):
            got = S.wait(t)
            vm = None
            if sub is not None:
                vm = np.zeros(g.n, np.uint8)
                vm[sub.astype(np.int64)] = 1
            want = oracle.topk(g.n, g.src, g.dst, g.w, k, p, vertex_mark=vm)
            assert_parity(got, want, p, ei, ctx=f"served k={k} p={p} subset={sub is not None}")


def test_admission_by_budget(tt, graph):
    g, G = graph
    with tt.Server(G, slots=4, scratch_budget=1) as S:
        with pytest.raises(tt.TopKError) as e:
            S.submit(10, 1.0)
        assert e.value.code == tt.TT_E_BUDGET
    need = None
    with tt.Server(G, slots=4, scratch_budget=1 << 40) as S:
        need = S.request_bytes(100)
        assert need > 0 and S.request_bytes(5000) > need and S.request_bytes(100, 1000) > need
    # room for one request at a time: four slots, but requests run one by one
    reqs = [(100, p, None) for p in P_CHOICES]
    with tt.Server(G, slots=4, scratch_budget=int(need * 1.5)) as S:
        tickets = [S.submit(k, p, sub) for k, p, sub in reqs]
        served = [S.wait(t) for t in tickets]
        info = S.info()
    assert info["max_running"] == 1 and info["peak_bytes"] <= int(need * 1.5)
    for (k, p, sub), b in zip(reqs, served):
        assert same(G.topk(k, p), b)


def test_scratch_held_stays_within_budget(tt, graph):
    """Workers keep their scratch between requests; the device bytes they actually hold (the
    allocator's live blocks) never exceed the budget, also after large and subset requests on
    several workers, and requests still all complete."""
    g, G = graph
    rng = np.random.default_rng(3)
    with tt.Server(G, slots=4, scratch_budget=1 << 40) as S:
        small, big, sub = S.request_bytes(50), S.request_bytes(8000), S.request_bytes(50, 1000)
    budget = 2 * big + sub
    reqs = []
    for t in range(40):
        k = int(rng.choice([20, 50, 8000]))
        subset = np.sort(rng.choice(g.n, size=1000, replace=False)).astype(np.uint32) if t % 5 == 0 else None
        reqs.append((k, float(P_CHOICES[t % len(P_CHOICES)]), subset))
    with tt.Server(G, slots=4, scratch_budget=budget) as S:
        tickets = [S.submit(k, p, sub) for k, p, sub in reqs]
        held_max = 0
        out = []
        for t in tickets:
            out.append(S.wait(t))
            held_max = max(held_max, S.scratch_bytes())
        info = S.info()
        held_end = S.scratch_bytes()
    log(f"budget {budget}, held max {held_max}, end {held_end}, peak charged {info['peak_bytes']}, small {small}")
    assert info["completed"] == len(reqs)
    assert held_max <= budget and held_end <= budget and info["peak_bytes"] <= budget
    for (k, p, sub), b in zip(reqs[:10], out[:10]):
        assert same(G.topk(k, p, subset=sub), b)


def test_poll_and_bad_requests(tt, graph):
    g, G = graph
    with tt.Server(G, slots=2, scratch_budget=8 << 30) as S:
        t = S.submit(50, 2.0)
        S.wait(t)
        with pytest.raises(tt.TopKError):
            S.submit(10, float("nan"))
        with pytest.raises(tt.TopKError) as e:
            S.submit(10, 1.0, subset=[g.n])
        assert e.value.code == tt.TT_E_VERTEX_RANGE
        t2 = S.submit(20, -math.inf)
        r = S.wait(t2)
        assert r["n_out"] == 20
        # the ticket was released by wait: polling or waiting again is refused, never blocks
        with pytest.raises(tt.TopKError) as e:
            S.done(t2)
        assert e.value.code == tt.TT_E_ARG
        with pytest.raises(ValueError):
            S.wait(t2)
        buf = (tt.Triangle * 32)()
        n_out = ctypes.c_uint32(0)
        assert tt.library().server_wait(S._h, t2, buf, ctypes.byref(n_out), None) == tt.TT_E_ARG
        assert tt.library().server_wait(S._h, 10**9, buf, ctypes.byref(n_out), None) == tt.TT_E_ARG
