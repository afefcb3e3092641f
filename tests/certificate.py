"""Complete parity checks on graphs too large for the oracle to enumerate whole (test
infrastructure; calls only numpy and the oracle).

Every weight of a triangle is at most its largest one, and m_p is non-decreasing in each
argument for every p in [-inf, +inf] (Eq. 1 and its limits), so a triangle scoring at least S,
with weights a >= b >= c and every graph weight <= W, has
    a >= S,
    b >= y(S) = the least b with m_p(W, b, b) >= S,
    c >= z(S) = the least c with m_p(W, W, c) >= S.
If S is at most the true k-th score, every triangle of the true top-k meets the three bounds, so
a subgraph H holding every triangle that meets them holds the true top-k, and the oracle's
top-k of H is the true top-k of the whole graph (H's other triangles are triangles of the graph
as well, ranked by the same total order).  Three such H:
  one-edge  : the edges of weight >= S, and every edge of weight >= z touching their ends (only
              the triangles on the edges of weight >= S are enumerated);
  two-edge  : the edges of weight >= max(y, z), and every edge of weight >= z that closes a
              wedge of two of them;
  all-edges : every edge of weight >= z.
certified_topk finds such an S from the oracle alone: the k-th score of k real triangles (those
on the graph's heaviest edges, or in the subgraph of its heaviest edges) can only be at most the
true k-th score.
"""
from __future__ import annotations

import math

import numpy as np

CHUNK = 1 << 26
SLACK = 1e-9  # relative: the bounds below are lowered by this much before flooring


def pair_keys(a, b):
    a = np.asarray(a, np.uint64)
    b = np.asarray(b, np.uint64)
    return (np.minimum(a, b) << np.uint64(32)) | np.maximum(a, b)


def bounds(p: float, S: float, W: int):
    """(a_min, y, z): integer lower bounds of the largest, second largest and smallest weight
    of any triangle with m_p >= S when every weight is <= W (conservative by SLACK)."""
    lo = lambda x: max(0, int(math.floor(x * (1.0 - SLACK))))  # noqa: E731
    a_min = lo(S)
    if p == math.inf:
        return a_min, 0, 0
    if p == -math.inf:
        return a_min, a_min, a_min
    if p == 0.0:  # a b c >= S^3
        return a_min, lo(math.sqrt(S ** 3 / W)), lo(S ** 3 / W ** 2)
    if p > 0:
        t, Wp = 3.0 * S ** p, float(W) ** p
        y = ((t - Wp) / 2.0) ** (1.0 / p) if t > Wp else 0.0
        z = (t - 2.0 * Wp) ** (1.0 / p) if t > 2.0 * Wp else 0.0
        return a_min, lo(y), lo(z)
    # p < 0: sum of w^p <= 3 S^p, each term positive
    t, Wp = 3.0 * S ** p, float(W) ** p
    y = ((t - Wp) / 2.0) ** (1.0 / p)
    z = (t - 2.0 * Wp) ** (1.0 / p)
    return a_min, lo(y), lo(z)


def _select(src, dst, w, mask_fn, log=None):
    parts = []
    for c, lo in enumerate(range(0, len(src), CHUNK)):
        idx = np.nonzero(mask_fn(src[lo:lo + CHUNK], dst[lo:lo + CHUNK], w[lo:lo + CHUNK]))[0]
        parts.append(idx + lo)
        if log and c % 8 == 7:
            log(f"    pass at edge {lo + CHUNK} of {len(src)}")
    return np.concatenate(parts) if parts else np.zeros(0, np.int64)


def _count(w, t):
    return int(sum(np.count_nonzero(w[lo:lo + CHUNK] >= t) for lo in range(0, len(w), CHUNK)))


def _wedge_pairs(a, b):
    """Unordered pairs {x, y} of vertices that are both joined to a common vertex by the
    edges (a, b), as sorted unique pair keys."""
    ends = np.concatenate([a, b]).astype(np.uint64)
    other = np.concatenate([b, a]).astype(np.uint64)
    order = np.argsort(ends, kind="stable")
    ends, other = ends[order], other[order]
    starts = np.flatnonzero(np.r_[True, ends[1:] != ends[:-1]])
    sizes = np.diff(np.r_[starts, len(ends)])
    keys = []
    for s, c in zip(starts[sizes > 1].tolist(), sizes[sizes > 1].tolist()):
        nb = other[s:s + c]
        iu, ju = np.triu_indices(c, 1)
        keys.append(pair_keys(nb[iu], nb[ju]))
    return np.unique(np.concatenate(keys)) if keys else np.zeros(0, np.uint64)


def subgraph(n, src, dst, w, p, S, W=None, max_wedges=50_000_000, form=None, log=None):
    """Edge indices of a subgraph H holding every triangle of score >= S (module docstring),
    and a description of the form used (`form` forces one; by default the smallest)."""
    say = log or (lambda msg: None)
    if W is None:
        W = int(max(int(w[lo:lo + CHUNK].max()) for lo in range(0, len(w), CHUNK)))
    a_min, y, z = bounds(p, S, W)
    n_all = _count(w, z) if z > 0 else len(w)
    n_two = _count(w, max(y, z)) if max(y, z) > 0 else len(w)
    n_heavy = _count(w, a_min)
    desc = {"p": p, "S": S, "W": W, "a_min": a_min, "y": y, "z": z, "heavy": n_heavy, "two": n_two, "all": n_all}
    say(f"  certificate bounds {desc}")
    if form is None:
        form = ("all-edges" if n_all <= 30_000_000 or (n_all <= n_two and n_all <= 20 * n_heavy) else
                "two-edge" if n_two <= 3_000_000 else "one-edge")
    if form == "all-edges":
        desc["form"] = "all-edges"
        return _select(src, dst, w, lambda s, d, ww: ww >= z), desc
    if form == "two-edge":
        B = _select(src, dst, w, lambda s, d, ww: ww >= max(y, z))
        wk = _wedge_pairs(src[B], dst[B])
        desc["wedges"] = int(len(wk))
        assert len(wk) <= max_wedges, desc
        # ends of the wedges' open pairs: an edge closes a wedge only if both its ends are such
        wend = np.zeros(n, np.bool_)
        wend[(wk >> np.uint64(32)).astype(np.int64)] = True
        wend[(wk & np.uint64(0xFFFFFFFF)).astype(np.int64)] = True

        def closes(s, d, ww):
            out = np.zeros(len(s), bool)
            cand = np.nonzero(wend[s] & wend[d] & (ww >= z))[0]
            if len(wk) and len(cand):
                k = pair_keys(s[cand], d[cand])
                pos = np.minimum(np.searchsorted(wk, k), len(wk) - 1)
                out[cand[wk[pos] == k]] = True
            return out

        say(f"  {len(B)} edges >= max(y, z), {len(wk)} wedges over {int(wend.sum())} vertices")
        C = _select(src, dst, w, closes, log=say)
        desc["form"] = "two-edge"
        return np.union1d(B, C), desc
    A = _select(src, dst, w, lambda s, d, ww: ww >= a_min)
    mark = np.zeros(n, np.bool_)
    mark[src[A]] = True
    mark[dst[A]] = True
    say(f"  {len(A)} edges >= {a_min}, {int(mark.sum())} of their ends")
    desc["form"] = "one-edge"
    return _select(src, dst, w, lambda s, d, ww: (ww >= z) & (mark[s] | mark[d]), log=say), desc


def _weights_desc_at(w, rank):
    """The weight at a rank (0 = heaviest) of the edge weights (numpy partition, chunk-free)."""
    rank = min(rank, len(w) - 1)
    return int(np.partition(w, len(w) - 1 - rank)[len(w) - 1 - rank])


def _oracle_topk(n, src, dst, w, sel, k, p, vertex_mark, edge_mark=None, nthreads=0):
    import oracle
    kw = {}
    if edge_mark is not None:
        kw = {"edge_mark": edge_mark, "from_marked_edges": True}
    return oracle.topk(n, src[sel], dst[sel], w[sel], k, p, nthreads=nthreads, vertex_mark=vertex_mark, **kw)


def certified_topk(n, src, dst, w, k, p, vertex_mark=None, log=None, nthreads=0, W=None):
    """The exact top-k (oracle.topk's result on the whole graph) computed by the oracle on a
    certified subgraph.  Returns (result, description)."""
    say = log or (lambda msg: None)
    if W is None:
        W = int(max(int(w[lo:lo + CHUNK].max()) for lo in range(0, len(w), CHUNK)))
    # step 1: a lower bound S1 of the true k-th score, from k real triangles
    S1, steps = None, []
    rank = 4 * max(k, 250)
    while S1 is None:
        t = _weights_desc_at(w, rank) if rank < len(w) else 1
        if p < 0:  # the subgraph of the heaviest edges (the answer's edges are all heavy)
            sel = _select(src, dst, w, lambda s, d, ww: ww >= t)
            r = _oracle_topk(n, src, dst, w, sel, k, p, vertex_mark, nthreads=nthreads)
        else:  # the triangles on the heaviest edges
            A = _select(src, dst, w, lambda s, d, ww: ww >= t)
            mark = np.zeros(n, np.bool_)
            mark[src[A]] = True
            mark[dst[A]] = True
            sel = _select(src, dst, w, lambda s, d, ww: mark[s] | mark[d])
            r = _oracle_topk(n, src, dst, w, sel, k, p, vertex_mark, edge_mark=(w[sel] >= t).astype(np.uint8),
                             nthreads=nthreads)
        steps.append({"t": t, "edges": int(len(sel)), "found": r["n_out"]})
        say(f"  lower bound step: weight >= {t}: {len(sel)} edges, {r['n_out']} triangles")
        if r["n_out"] == k:
            S1 = float(r["score"][-1])
        elif t <= 1:  # the whole graph holds fewer than k triangles: this is the answer
            return r, {"form": "whole graph", "steps": steps}
        else:
            rank *= 8
    # step 2: the subgraph holding every triangle that scores >= S1
    sel, desc = subgraph(n, src, dst, w, p, S1, W=W, log=say)
    desc["steps"] = steps
    say(f"  certificate {desc['form']}: S1={S1}, {len(sel)} edges")
    if desc["form"] == "one-edge":
        r = _oracle_topk(n, src, dst, w, sel, k, p, vertex_mark,
                         edge_mark=(w[sel] >= desc["a_min"]).astype(np.uint8), nthreads=nthreads)
    else:
        r = _oracle_topk(n, src, dst, w, sel, k, p, vertex_mark, nthreads=nthreads)
    desc["edges"] = int(len(sel))
    return r, desc
