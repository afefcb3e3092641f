"""CPU property tests of the library's pruning bounds (the bound of Sec. 3.2, generalised to
every p through the monotonicity of m_p in each weight, Eq. 1): the host build of the very
functions the kernels call (csrc/enum.h, compiled by tests/bounds_shim.hip) must never exclude
a triangle whose order key reaches the band's lower bound L.

For a triangle on entry u->v with weights a = w_uv, x = w_uc <= maxw(u), y = w_vc <= maxw(v),
every weight <= W, and key(a, x, y) >= L:
  * the entry filter passes:        bound_ok(L, a, maxw(u), maxw(v))
  * the row floors admit both:      x >= min_other(L, a, maxw(v)),  y >= min_other(L, a, maxw(u))
  * the lightest edge reaches:      min(a, x, y) >= weight_floor(L, W)
  * the row / order streams hold it: score_floor(L) <= m_p(a, x, y) <= entry_bound(a, maxw(u), maxw(v))
checked on random triples (ties, log-uniform weights, weights near 2^32 - 1, mixed extremes), with
L at the triangle's own key (the boundary case), just below it, and at other triangles' keys,
for p = +-inf, +-50, |p| <= 1e-6, and the usual means."""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SHIM = os.path.join(HERE, "bounds_shim.hip")

P_VALUES = [math.inf, -math.inf, 1.0, 2.0, 0.0, 0.5, -1.0, 3.0, -3.0, 50.0, -50.0, 1e-7, -1e-7, 1e-6, -1e-6,
            0.999999, 1.000001, 1.7, -0.3]
U32 = 2**32 - 1


@pytest.fixture(scope="module")
def bt(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("bt") / "libbt.so")
    subprocess.run(["hipcc", "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", "-fPIC", "-shared",
                    "-ffp-contract=off", "-w", "-o", out, SHIM], check=True)
    lib = ctypes.CDLL(out)
    u32, u64, dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    p64 = ctypes.POINTER(ctypes.c_uint64)
    lib.bt_key.argtypes = [dbl, u32, u32, u32, p64, p64]
    lib.bt_key.restype = None
    lib.bt_score.argtypes = [dbl, u64, u64]
    lib.bt_score.restype = dbl
    lib.bt_bound_ok.argtypes = [dbl, u64, u64, u32, u32, u32]
    lib.bt_bound_ok.restype = ctypes.c_int
    lib.bt_min_other.argtypes = [dbl, u64, u64, u32, u32]
    lib.bt_min_other.restype = u64
    lib.bt_weight_floor.argtypes = [dbl, u64, u64, u32]
    lib.bt_weight_floor.restype = u64
    lib.bt_score_floor.argtypes = [dbl, u64, u64]
    lib.bt_score_floor.restype = u64
    lib.bt_entry_bound.argtypes = [dbl, u32, u32, u32]
    lib.bt_entry_bound.restype = u32
    return lib


def key(lib, p, a, b, c):
    hi, lo = ctypes.c_uint64(), ctypes.c_uint64()
    lib.bt_key(p, a, b, c, ctypes.byref(hi), ctypes.byref(lo))
    return (hi.value << 64) | lo.value


def split(L):
    return L >> 64, L & (2**64 - 1)


def triples(rng, kind, n):
    if kind == "ties":
        w = rng.integers(1, 21, (n, 3))
    elif kind == "loguniform":
        w = np.exp(rng.uniform(0, math.log(U32), (n, 3))).astype(np.int64) + 1
    elif kind == "near_max":
        w = U32 - rng.integers(0, 1000, (n, 3))
    else:  # mixed extremes: one light weight, two near the top
        w = np.stack([rng.integers(1, 50, n), U32 - rng.integers(0, 10**6, n), U32 - rng.integers(0, 10**6, n)], 1)
        w = np.take_along_axis(w, rng.permuted(np.tile(np.arange(3), (n, 1)), axis=1), 1)
    return np.minimum(w, U32).astype(np.int64)


def row_maxima(rng, x, y, kind):
    """maxw(u) >= x and maxw(v) >= y (sometimes equal, sometimes the top weight)."""
    def up(v):
        r = rng.random()
        if r < 0.4:
            return int(v)
        if r < 0.6:
            return U32
        return int(min(U32, v + rng.integers(0, max(2, v))))
    return up(x), up(y)


@pytest.mark.parametrize("p", P_VALUES)
@pytest.mark.parametrize("kind", ["ties", "loguniform", "near_max", "mixed"])
def test_no_qualifying_triangle_is_pruned(bt, p, kind):
    rng = np.random.default_rng(hash((p, kind)) & 0xFFFFFFFF)
    T = triples(rng, kind, 1500)
    keys = [key(bt, p, int(a), int(x), int(y)) for a, x, y in T]
    bad = []
    for t, (a, x, y) in enumerate(T.tolist()):
        K = keys[t]
        Wu, Wv = row_maxima(rng, x, y, kind)
        W = max(a, Wu, Wv, int(rng.choice([max(a, Wu, Wv), U32])))
        score = bt.bt_score(p, *split(K))
        Ls = {K, max(K - 1, 1), keys[int(rng.integers(0, len(keys)))], keys[int(rng.integers(0, len(keys)))]}
        for L in Ls:
            if L > K:
                continue
            Lh, Ll = split(L)
            if not bt.bt_bound_ok(p, Lh, Ll, a, Wu, Wv):
                bad.append(("bound_ok", a, x, y, Wu, Wv, L))
            if x < bt.bt_min_other(p, Lh, Ll, a, Wv):
                bad.append(("min_other x", a, x, y, Wv, L, bt.bt_min_other(p, Lh, Ll, a, Wv)))
            if y < bt.bt_min_other(p, Lh, Ll, a, Wu):
                bad.append(("min_other y", a, x, y, Wu, L, bt.bt_min_other(p, Lh, Ll, a, Wu)))
            if min(a, x, y) < bt.bt_weight_floor(p, Lh, Ll, W):
                bad.append(("weight_floor", a, x, y, W, L, bt.bt_weight_floor(p, Lh, Ll, W)))
            sf = bt.bt_score_floor(p, Lh, Ll)
            if sf > score:
                bad.append(("score_floor", a, x, y, L, sf, score))
            eb = bt.bt_entry_bound(p, a, Wu, Wv)
            if eb < sf or eb < math.floor(score) or eb > max(a, Wu, Wv):
                bad.append(("entry_bound", a, x, y, Wu, Wv, eb, sf, score))
        if len(bad) > 20:
            break
    assert not bad, bad[:10]


@pytest.mark.parametrize("p", P_VALUES)
def test_keys_order_like_the_scores(bt, p):
    """The order key is a monotone transform of m_p: key(t1) > key(t2) implies score(t1) >=
    score(t2), and equal keys give equal scores."""
    rng = np.random.default_rng(7)
    T = np.concatenate([triples(rng, k, 400) for k in ("ties", "loguniform", "near_max", "mixed")])
    ks = [key(bt, p, int(a), int(b), int(c)) for a, b, c in T]
    sc = [bt.bt_score(p, *split(k)) for k in ks]
    order = np.argsort(np.array([float(k) for k in ks]), kind="stable")
    pairs = sorted(zip(ks, sc))
    for (k1, s1), (k2, s2) in zip(pairs, pairs[1:]):
        assert s1 <= s2 and (k1 != k2 or s1 == s2), (p, k1, s1, k2, s2)
    assert len(order) == len(T)
