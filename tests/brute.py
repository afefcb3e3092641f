"""Pure-Python brute force on tiny graphs, used to pin the oracle (not the oracle itself).

Everything here enumerates all vertex triples and ranks them with exact rational arithmetic
where the mean allows it, so it shares no code or algorithm with ``oracle/``.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction


def edge_dict(src, dst, w):
    d = {}
    for a, b, x in zip(src, dst, w):
        a, b = int(a), int(b)
        d[(min(a, b), max(a, b))] = int(x)
    return d


def all_triangles(n, src, dst, w):
    """[(i, j, l, w_ij, w_il, w_jl)] over all triples i<j<l whose three pairs are edges."""
    E = edge_dict(src, dst, w)
    out = []
    for i, j, l in itertools.combinations(range(n), 3):
        a, b, c = E.get((i, j)), E.get((i, l)), E.get((j, l))
        if a is not None and b is not None and c is not None:
            out.append((i, j, l, a, b, c))
    return out


def exact_rank_value(p, a, b, c):
    """A value that orders triangles exactly like m_p, for p in {-inf, 0, 1, 2, +inf}."""
    if p == math.inf:
        return max(a, b, c)
    if p == -math.inf:
        return min(a, b, c)
    if p == 1:
        return Fraction(a + b + c, 3)
    if p == 2:
        return a * a + b * b + c * c
    if p == 0:
        return a * b * c
    raise ValueError(p)


def float_mean(p, a, b, c):
    """m_p in floating point straight from Eq. 1 (for generic p)."""
    return ((a ** p + b ** p + c ** p) / 3.0) ** (1.0 / p)


def topk(n, src, dst, w, k, p):
    """Brute-force top-k: all triangles sorted by (value desc, i, j, l)."""
    tris = all_triangles(n, src, dst, w)
    if p in (math.inf, -math.inf, 0, 1, 2):
        keyf = lambda t: (-exact_rank_value(p, t[3], t[4], t[5]), t[0], t[1], t[2])
    else:
        keyf = lambda t: (-float_mean(p, t[3], t[4], t[5]), t[0], t[1], t[2])
    tris.sort(key=keyf)
    return tris[:k], len(tris)
