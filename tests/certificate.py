"""Complete parity checks on graphs too large for the oracle to enumerate whole (test
infrastructure; calls only numpy and, in the tests, the oracle).

Every weight of a triangle is at most its largest one, and m_p is non-decreasing in each
argument for every p in [-inf, +inf] (Eq. 1 and its limits), so a triangle scoring at least S,
with weights a >= b >= c and every graph weight <= W, has
    a >= S,
    b >= y(S) = the least b with m_p(W, b, b) >= S,
    c >= z(S) = the least c with m_p(W, W, c) >= S.
Let S be the k-th score the GPU returned.  Its k triangles are real (checked separately), so
S is at most the true k-th score, and every triangle of the true top-k satisfies the three
bounds with this S.  A subgraph H that holds every triangle meeting the bounds therefore holds
the true top-k, and the oracle's top-k of H is the true top-k of the whole graph (H's other
triangles are triangles of the graph as well, ranked by the same total order).  Three such H:
  one-edge  : the edges of weight >= S, and every edge of weight >= z touching their ends;
  two-edge  : the edges of weight >= max(y, z), and every edge of weight >= z that closes a
              wedge of two of them;
  all-edges : every edge of weight >= z.
The smallest is used.
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


def _select(src, dst, w, mask_fn):
    parts = []
    for lo in range(0, len(src), CHUNK):
        idx = np.nonzero(mask_fn(src[lo:lo + CHUNK], dst[lo:lo + CHUNK], w[lo:lo + CHUNK]))[0]
        parts.append(idx + lo)
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


def subgraph(n, src, dst, w, p, S, W=None, max_wedges=50_000_000, form=None):
    """Edge indices of a subgraph H holding every triangle of score >= S (module docstring),
    and a description of the form used (`form` forces one; by default the smallest)."""
    if W is None:
        W = int(max(int(w[lo:lo + CHUNK].max()) for lo in range(0, len(w), CHUNK)))
    a_min, y, z = bounds(p, S, W)
    n_all = _count(w, z) if z > 0 else len(w)
    n_two = _count(w, max(y, z)) if max(y, z) > 0 else len(w)
    n_heavy = _count(w, a_min)
    desc = {"p": p, "S": S, "W": W, "a_min": a_min, "y": y, "z": z, "heavy": n_heavy, "two": n_two, "all": n_all}
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

        def closes(s, d, ww):
            if not len(wk):
                return np.zeros(len(s), bool)
            k = pair_keys(s, d)
            pos = np.minimum(np.searchsorted(wk, k), len(wk) - 1)
            return (ww >= z) & (wk[pos] == k)

        C = _select(src, dst, w, closes)
        desc["form"] = "two-edge"
        return np.union1d(B, C), desc
    A = _select(src, dst, w, lambda s, d, ww: ww >= a_min)
    mark = np.zeros(n, np.bool_)
    mark[src[A]] = True
    mark[dst[A]] = True
    desc["form"] = "one-edge"
    return _select(src, dst, w, lambda s, d, ww: (ww >= z) & (mark[s] | mark[d])), desc
