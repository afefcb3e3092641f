"""The served form at the serving workload's full size: a resident Chung-Lu graph with 10M
vertices and ~200M edges (gamma 2.1, Zipf(1.8) weights) and the Poisson request mix (k
log-uniform in [10, 1e4], p from {-inf, -1, 0, 1, 2, +inf}, 20% restricted to 1,000-vertex
subsets).  Every served result must equal the single-query result of the same request, and a
sample of requests, one per p plus subset requests, must equal the oracle's answer, computed by
the oracle alone on a subgraph that provably holds it (tests/certificate.py)."""
import math
import sys
import time

import numpy as np
import pytest

import certificate
import graphgen
import oracle
from paritylib import EdgeIndex, assert_parity, triples

pytestmark = pytest.mark.gpu

N_REQ = 64


def log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def served():
    import torch
    import paper_1910_00692_amd as tt
    g = graphgen.serve_graph()
    log(f"serve graph n={g.n} m={g.m}")
    dev = torch.device("cuda:0")
    s = torch.from_numpy(g.src.view(np.int32)).to(dev)
    d = torch.from_numpy(g.dst.view(np.int32)).to(dev)
    w = torch.from_numpy(g.w.view(np.int32)).to(dev)
    G = tt.Graph(g.n, s, d, w, stream=torch.cuda.current_stream(dev))
    del s, d, w
    reqs = graphgen.query_stream(N_REQ, g.n, seed=3)
    singles = [G.topk(r["k"], r["p"], subset=r["subset"]) for r in reqs]
    log("single-query results done")
    with tt.Server(G, slots=8, scratch_budget=16 << 30) as S:
        start = time.perf_counter()
        tickets = []
        for r in reqs:  # submitted at their Poisson arrival times
            now = time.perf_counter() - start
            if r["t"] > now:
                time.sleep(r["t"] - now)
            tickets.append(S.submit(r["k"], r["p"], r["subset"]))
        out = [S.wait(t) for t in tickets]
        info = S.info()
    log(f"server info {info}")
    G.close()
    yield g, reqs, singles, out, info


def test_served_equals_single_full_size(served):
    g, reqs, singles, out, info = served
    assert info["completed"] == len(reqs)
    for r, a, b in zip(reqs, singles, out):
        assert a["n_out"] == b["n_out"] and triples(a) == triples(b) and np.array_equal(a["score"], b["score"]), \
            (r["k"], r["p"], r["subset"] is not None)
    assert info["max_running"] >= 2


def pick_for_oracle(reqs):
    """One request per p (the smallest k of that p, to bound the oracle's work) and two subset
    requests."""
    chosen = []
    for p in graphgen.P_CHOICES:
        c = [t for t, r in enumerate(reqs) if r["p"] == p and r["subset"] is None]
        if c:
            chosen.append(min(c, key=lambda t: reqs[t]["k"]))
    subs = sorted((t for t, r in enumerate(reqs) if r["subset"] is not None), key=lambda t: reqs[t]["k"])
    return chosen + subs[:2]


def test_served_against_oracle_full_size(served):
    g, reqs, _, out, _ = served
    picked = pick_for_oracle(reqs)
    assert len(picked) >= 6 and any(reqs[t]["subset"] is not None for t in picked)
    assert {-1.0, 0.0} <= {reqs[t]["p"] for t in picked}
    W = int(g.w.max())
    ei = EdgeIndex(g.src, g.dst, g.w)
    for t in picked:
        r, got = reqs[t], out[t]
        k, p = r["k"], r["p"]
        vm = None
        if r["subset"] is not None:
            vm = np.zeros(g.n, np.uint8)
            vm[r["subset"].astype(np.int64)] = 1
        t0 = time.time()
        want, desc = certificate.certified_topk(g.n, g.src, g.dst, g.w, k, p, vertex_mark=vm, W=W)
        log(f"request {t}: k={k} p={p} subset={vm is not None}: {desc.get('form')} {desc.get('edges')} edges "
            f"({time.time() - t0:.1f}s)")
        assert_parity(got, want, p, ei, ctx=f"served request {t} k={k} p={p}")
