// sampling.hip — the paper's other two triangle samplers on the device: weighted wedge sampling
// (Alg. 4, Eqs. wedgeone-wedgethree, Prop. 2) and weighted path sampling (Alg. 5, Eqs.
// pathone-paththree, Prop. 3).  Both draw small subgraphs with probabilities built from the
// edge weights raised to the sampling exponent q, keep the draws that close a triangle, and
// return the top-k of the distinct triangles found, by the true m_p.
//
// Every draw is an inverse-CDF choice, so the device tables are prefix sums: over the
// symmetric adjacency (rows sorted by neighbour) the running sum P_a(t) of w^q along the row of
// a, and, per scheme, the prefix over vertices of the wedge weight 2 d_a D(a) or over directed
// entries of the path weight of Eq. pathone.  Each conditional distribution of a draw is of the
// form weight(t) = alpha w_t^q + beta along one row (with one entry left out for paths), whose
// cumulative alpha P_a(t) + beta (t + 1) is searched directly.
//
// Draw s uses the SplitMix64 outputs 3s, 3s+1, 3s+2 (Steele, Lea, Flood 2014) of the seed as
// its three uniforms (x >> 11) 2^-53; the tables are FP64.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstring>

#include "common.h"
#include "enum.h"
#include "scan.h"

namespace {

constexpr uint64_t EMPTY_KEY = ~0ull;
constexpr uint32_t PACK_BITS = 21; // a triangle (i < j < l) packed in 63 bits: n <= 2^21

__device__ __forceinline__ uint64_t mix_at(uint64_t seed, uint64_t s) {
    uint64_t z = seed + (s + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }
__device__ __forceinline__ double powq(uint32_t w, double q) { return q == 1.0 ? (double)w : pow((double)w, q); }

// Both directions of every oriented entry, as (row << 32 | neighbour) keys with the weight.
__global__ __launch_bounds__(256) void k_sym_keys(const uint32_t *osrc, const uint32_t *col, const uint32_t *wgt,
                                                  uint64_t m, uint64_t *keys, uint32_t *vals) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t u = osrc[e], v = col[e];
        const uint32_t w = wgt[e];
        keys[2 * e] = (u << 32) | v;
        keys[2 * e + 1] = (v << 32) | u;
        vals[2 * e] = w;
        vals[2 * e + 1] = w;
    }
}

__global__ __launch_bounds__(256) void k_sym_cols(const uint64_t *keys, uint64_t N, uint32_t *scol) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
        scol[i] = (uint32_t)keys[i];
}

// P_a(t): the inclusive sum of w^q along each row (one wave per row, 64 entries at a time).
__global__ __launch_bounds__(256) void k_row_prefix(const uint64_t *srstart, const uint32_t *sw, uint32_t n, double q,
                                                    double *out) {
    const int lane = threadIdx.x & 63;
    const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t v = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; v < n; v += nw) {
        const uint64_t lo = srstart[v], hi = srstart[v + 1];
        double carry = 0.0;
        for (uint64_t t0 = lo; t0 < hi; t0 += 64) {
            const uint64_t t = t0 + lane;
            const double x = t < hi ? powq(sw[t], q) : 0.0;
            const double incl = wave_incl_scan(x) + carry;
            if (t < hi) out[t] = incl;
            carry = __shfl(incl, 63, 64);
        }
    }
}

__device__ __forceinline__ double row_total(const uint64_t *srstart, const double *rowp, uint32_t v) {
    const uint64_t lo = srstart[v], hi = srstart[v + 1];
    return hi > lo ? rowp[hi - 1] : 0.0;
}

// Eq. wedgeone: W1(a) = 2 d_a D(a).
__global__ __launch_bounds__(256) void k_wedge_vw(const uint64_t *srstart, const double *rowp, uint32_t n, double *vw) {
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
        vw[v] = 2.0 * (double)(srstart[v + 1] - srstart[v]) * row_total(srstart, rowp, (uint32_t)v);
}

// Eq. pathone for the directed entry a -> b (each edge appears in both rows):
//   (d_a - 1)(d_b - 1) w_ab^q + (d_a - 1)(D(b) - w_ab^q) + (d_b - 1)(D(a) - w_ab^q).
__global__ __launch_bounds__(256) void k_path_ew(const uint64_t *srstart, const uint32_t *scol, const uint32_t *sw,
                                                 const double *rowp, uint32_t n, double q, double *ew) {
    const int lane = threadIdx.x & 63;
    const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t a = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; a < n; a += nw) {
        const uint64_t lo = srstart[a], hi = srstart[a + 1];
        const double da = (double)(hi - lo) - 1.0, Da = hi > lo ? rowp[hi - 1] : 0.0;
        for (uint64_t t = lo + lane; t < hi; t += 64) {
            const uint32_t b = scol[t];
            const double wq = powq(sw[t], q);
            const double db = (double)(srstart[b + 1] - srstart[b]) - 1.0;
            const double Db = row_total(srstart, rowp, b);
            ew[t] = da * db * wq + da * (Db - wq) + db * (Da - wq);
        }
    }
}

// First t in [lo, hi) whose cumulative weight C(t) exceeds r (the last one if rounding leaves
// none).  C is non-decreasing.
template <typename C> __device__ __forceinline__ uint64_t first_over(uint64_t lo, uint64_t hi, double r, C cum) {
    uint64_t a = lo, b = hi;
    while (a < b) {
        const uint64_t mid = (a + b) >> 1;
        if (cum(mid) > r) b = mid; else a = mid + 1;
    }
    return a < hi ? a : hi - 1;
}

// Position of neighbour c in the sorted row [lo, hi), or ~0.
__device__ __forceinline__ uint64_t find_pos(const uint32_t *scol, uint64_t lo, uint64_t hi, uint32_t c) {
    uint64_t a = lo, b = hi;
    while (a < b) {
        const uint64_t mid = (a + b) >> 1;
        if (scol[mid] < c) a = mid + 1; else b = mid;
    }
    return a < hi && scol[a] == c ? a : ~0ull;
}

__device__ __forceinline__ uint64_t pack3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    return ((uint64_t)a << (2 * PACK_BITS)) | ((uint64_t)b << PACK_BITS) | c;
}

struct SymArgs {
    const uint64_t *srstart;
    const uint32_t *scol, *sw;
    const double *rowp;
    uint32_t n;
    double q;
};

// Alg. 4: a by Eq. wedgeone (vpre: inclusive prefix of W1 over vertices), b in N(a) by Eq.
// wedgetwo (weight d_a w_ab^q + D(a)), c in N(a) by Eq. wedgethree (weight w_ac^q + w_ab^q); the
// draw closes a triangle when c != b and {b, c} is an edge.
__global__ __launch_bounds__(256) void k_wedge_draw(SymArgs S, const double *vpre, uint64_t budget, uint64_t seed,
                                                    uint64_t *keys, uint4 *wts, uint32_t *dump) {
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < budget; s += (uint64_t)gridDim.x * blockDim.x) {
        const double Z1 = vpre[S.n - 1];
        const double r0 = unit(mix_at(seed, 3 * s)) * Z1;
        const uint32_t a = (uint32_t)first_over(0, S.n, r0, [&](uint64_t v) { return vpre[v]; });
        const uint64_t lo = S.srstart[a], hi = S.srstart[a + 1];
        if (hi == lo) { // only reachable through rounding at the very end of the prefix
            keys[s] = EMPTY_KEY;
            if (dump) dump[4 * s] = a, dump[4 * s + 1] = dump[4 * s + 2] = ~0u, dump[4 * s + 3] = 0u;
            continue;
        }
        const double d = (double)(hi - lo), D = S.rowp[hi - 1];
        const double r1 = unit(mix_at(seed, 3 * s + 1)) * (2.0 * d * D);
        const uint64_t tb = first_over(lo, hi, r1, [&](uint64_t t) { return d * S.rowp[t] + (double)(t - lo + 1) * D; });
        const uint32_t b = S.scol[tb], wab = S.sw[tb];
        const double wq = powq(wab, S.q);
        const double r2 = unit(mix_at(seed, 3 * s + 2)) * (D + d * wq);
        const uint64_t tc = first_over(lo, hi, r2, [&](uint64_t t) { return S.rowp[t] + (double)(t - lo + 1) * wq; });
        const uint32_t c = S.scol[tc], wac = S.sw[tc];
        uint64_t key = EMPTY_KEY;
        uint32_t wbc = 0;
        if (tc != tb) {
            const uint64_t tbc = find_pos(S.scol, S.srstart[b], S.srstart[b + 1], c);
            if (tbc != ~0ull) {
                wbc = S.sw[tbc];
                key = pack3(a, b, c);
            }
        }
        keys[s] = key;
        wts[s] = make_uint4(wab, wac, wbc, 0u);
        if (dump) {
            dump[4 * s] = a;
            dump[4 * s + 1] = b;
            dump[4 * s + 2] = c;
            dump[4 * s + 3] = key != EMPTY_KEY ? 1u : 0u;
        }
    }
}

// The row holding entry t: the last v with srstart[v] <= t.
__device__ __forceinline__ uint32_t row_of(const uint64_t *srstart, uint32_t n, uint64_t t) {
    uint32_t lo = 0, hi = n; // srstart[lo] <= t < srstart[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (srstart[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Alg. 5: the directed entry a -> b by Eq. pathone (epre: inclusive prefix over entries), c in
// N(a) \ b by Eq. pathtwo (weight (d_b - 1)(w_ac^q + w_ab^q) + D(b) - w_ab^q), c' in N(b) \ a by
// Eq. paththree (weight w_ac^q + w_ab^q + w_bc'^q); the draw closes a triangle when c' = c.
__global__ __launch_bounds__(256) void k_path_draw(SymArgs S, const double *epre, uint64_t N, uint64_t budget,
                                                   uint64_t seed, uint64_t *keys, uint4 *wts, uint32_t *dump) {
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < budget; s += (uint64_t)gridDim.x * blockDim.x) {
        const double r0 = unit(mix_at(seed, 3 * s)) * epre[N - 1];
        const uint64_t t0 = first_over(0, N, r0, [&](uint64_t t) { return epre[t]; });
        const uint32_t a = row_of(S.srstart, S.n, t0), b = S.scol[t0], wab = S.sw[t0];
        const uint64_t la = S.srstart[a], ha = S.srstart[a + 1], lb = S.srstart[b], hb = S.srstart[b + 1];
        const double wq = powq(wab, S.q);
        const double dtb = (double)(hb - lb) - 1.0;
        const double Dtb = S.rowp[hb - 1] - wq; // D(b) - w_ab^q
        // c: cumulative over a's row with entry t0 (b) left out
        const double skip_c = dtb * (wq + wq) + Dtb;
        const double Z2 = ((double)(ha - la) - 1.0) * dtb * wq + ((double)(ha - la) - 1.0) * Dtb +
                          dtb * (S.rowp[ha - 1] - wq);
        const double r1 = unit(mix_at(seed, 3 * s + 1)) * Z2;
        const uint64_t tc = first_over(la, ha, r1, [&](uint64_t t) {
            const double cnt = (double)(t - la + 1);
            return dtb * (S.rowp[t] + cnt * wq) + cnt * Dtb - (t >= t0 ? skip_c : 0.0);
        });
        const uint32_t c = S.scol[tc], wac = S.sw[tc];
        const double wcq = powq(wac, S.q);
        // c': cumulative over b's row with the entry of a left out
        const uint64_t tab = find_pos(S.scol, lb, hb, a);
        const double skip_cp = wcq + wq + wq;
        const double Z3 = dtb * (wcq + wq) + Dtb;
        const double r2 = unit(mix_at(seed, 3 * s + 2)) * Z3;
        const uint64_t tcp = first_over(lb, hb, r2, [&](uint64_t t) {
            const double cnt = (double)(t - lb + 1);
            return cnt * (wcq + wq) + S.rowp[t] - (t >= tab ? skip_cp : 0.0);
        });
        const uint32_t cp = S.scol[tcp];
        uint64_t key = EMPTY_KEY;
        uint32_t wbc = 0;
        if (cp == c && c != b && tc != t0) {
            wbc = S.sw[tcp];
            key = pack3(a, b, c);
        }
        keys[s] = key;
        wts[s] = make_uint4(wab, wac, wbc, 0u);
        if (dump) {
            dump[4 * s] = a;
            dump[4 * s + 1] = b;
            dump[4 * s + 2] = c;
            dump[4 * s + 3] = cp;
        }
    }
}

__device__ __forceinline__ uint64_t hash64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xFF51AFD7ED558CCDull;
    x ^= x >> 33;
    x *= 0xC4CEB9FE1A85EC53ull;
    return x ^ (x >> 33);
}

// The distinct triangles of the draws (a hash set of packed triples), each appended once as a
// record scored by m_p; *count receives their number.
// count[1] receives the number of draws that closed a triangle.
__global__ __launch_bounds__(256) void k_tri_distinct(const uint64_t *keys, const uint4 *wts, uint64_t budget,
                                                      unsigned long long *table, uint64_t tmask, int mode, double p,
                                                      trec *out, unsigned long long *count) {
    unsigned long long hits = 0;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < budget; s += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[s];
        if (k == EMPTY_KEY) continue;
        hits++;
        uint64_t h = hash64(k) & tmask;
        for (;;) {
            const unsigned long long old = atomicCAS(&table[h], (unsigned long long)EMPTY_KEY, (unsigned long long)k);
            if (old == EMPTY_KEY) {
                const uint4 w = wts[s];
                const u128 key = score_key(mode, p, w.x, w.y, w.z);
                trec r;
                r.khi = (uint64_t)(key >> 64);
                r.klo = (uint64_t)key;
                r.i = (uint32_t)(k >> (2 * PACK_BITS));
                r.j = (uint32_t)(k >> PACK_BITS) & ((1u << PACK_BITS) - 1);
                r.l = (uint32_t)k & ((1u << PACK_BITS) - 1);
                r.pad = 0;
                out[atomicAdd(count, 1ull)] = r;
                break;
            }
            if (old == k) break;
            h = (h + 1) & tmask;
        }
    }
    hits = wave_sum(hits);
    if ((threadIdx.x & 63) == 0 && hits) atomicAdd(&count[1], hits);
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

unsigned grid_of(uint64_t items) {
    const uint64_t b = (items + 255) / 256, cap = (uint64_t)num_cus() * 16;
    return (unsigned)std::max<uint64_t>(1, std::min(b, cap));
}

} // namespace

// The symmetric adjacency (built once): both directions of every entry, sorted by (row,
// neighbour) with a device radix sort.
int ensure_sym(tt_graph *g, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g->init_mu);
    if (g->srstart) return TT_OK;
    const uint64_t m = g->m, N = 2 * m, nn = (uint64_t)g->n + 1;
    if (N >= (1ull << 31)) return fail(TT_E_TOO_LARGE, "the symmetric adjacency needs 2m < 2^31");
    int rc;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    uint64_t *srstart = nullptr;
    uint32_t *scol = nullptr, *sw = nullptr;
    struct Guard {
        std::vector<void *> p;
        hipStream_t s;
        ~Guard() {
            (void)hipStreamSynchronize(s);
            for (void *x : p) dev_free(nullptr, x, 0);
        }
    } guard{{}, s};
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                           (uint32_t *)nullptr, (uint32_t *)nullptr, (int)N, 0, 64, s) != hipSuccess)
        return fail(TT_E_DEVICE, "radix sort size query failed");
    if ((rc = dev_alloc(nullptr, (void **)&k0, N * 8 + 8)) || (guard.p.push_back(k0), false) ||
        (rc = dev_alloc(nullptr, (void **)&k1, N * 8 + 8)) || (guard.p.push_back(k1), false) ||
        (rc = dev_alloc(nullptr, (void **)&v0, N * 4 + 4)) || (guard.p.push_back(v0), false) ||
        (rc = dev_alloc(nullptr, &tmp, tmp_bytes + 16)) || (guard.p.push_back(tmp), false))
        return rc;
    if ((rc = dev_alloc(g, (void **)&srstart, (nn + 1) * 8)) || (rc = dev_alloc(g, (void **)&scol, N * 4 + 4)) ||
        (rc = dev_alloc(g, (void **)&sw, N * 4 + 4))) {
        dev_free(g, srstart, 0);
        dev_free(g, scol, 0);
        dev_free(g, sw, 0);
        return rc;
    }
    if (m) k_sym_keys<<<grid_of(m), 256, 0, s>>>(g->osrc, g->col, g->wgt, m, k0, v0);
    if (N && hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, k0, k1, v0, sw, (int)N, 0, 64, s) != hipSuccess) {
        dev_free(g, srstart, 0);
        dev_free(g, scol, 0);
        dev_free(g, sw, 0);
        return fail(TT_E_DEVICE, "radix sort failed");
    }
    if (N) k_sym_cols<<<grid_of(N), 256, 0, s>>>(k1, N, scol);
    if ((rc = exclusive_scan_u32_to_u64(g->deg, srstart, nn, s, nullptr))) return rc;
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    g->scol = scol;
    g->sw = sw;
    g->srstart = srstart;
    return TT_OK;
}

extern "C" int sample_triangles_by(tt_graph *g, int scheme, uint32_t k, double p, uint64_t budget, uint64_t seed,
                                   double qexp, uint32_t *draws, tt_triangle *out, uint32_t *n_out,
                                   tt_sampler_stats *stats) {
    if (n_out) *n_out = 0;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!g || !n_out) return fail(TT_E_ARG, "graph or n_out is NULL");
    if (scheme != TT_SAMPLE_WEDGE && scheme != TT_SAMPLE_PATH) return fail(TT_E_ARG, "unknown sampling scheme");
    if (std::isnan(p)) return fail(TT_E_ARG, "p is NaN");
    if (k && !out) return fail(TT_E_ARG, "out is NULL");
    if (!std::isnan(qexp) && !(qexp > 0.0 && std::isfinite(qexp)))
        return fail(TT_E_ARG, "the sampling exponent q must be finite and > 0 (or NaN for the default)");
    if (g->n > (1u << 21)) return fail(TT_E_TOO_LARGE, "wedge and path sampling take graphs of at most 2^21 vertices");
    if (budget == 0 || g->m == 0 || (k == 0 && !draws)) { set_error(""); return TT_OK; }
    if (budget > (1ull << 31)) return fail(TT_E_TOO_LARGE, "budget must be <= 2^31");
    if (std::isnan(qexp)) qexp = (std::isfinite(p) && p > 0.0) ? p : 1.0;
    std::lock_guard<std::mutex> lock(g->mu);
    (void)hipSetDevice(g->device);
    QueryCtx *q = &g->q;
    hipStream_t s = q->stream;
    int rc;
    if ((rc = ensure_sym(g, s))) return rc;
    const uint64_t N = 2 * g->m;
    if (g->srow_q != qexp) {
        if (!g->srowp && (rc = dev_alloc(g, (void **)&g->srowp, N * 8 + 8))) return rc;
        g->srow_q = -1.0;
        k_row_prefix<<<grid_of((uint64_t)g->n * 64), 256, 0, s>>>(g->srstart, g->sw, g->n, qexp, g->srowp);
        HIP_TRY(hipGetLastError());
        g->srow_q = qexp;
    }
    const uint64_t items = scheme == TT_SAMPLE_WEDGE ? g->n : N;
    uint64_t tbits = 1;
    while ((1ull << tbits) < 2 * budget) tbits++;
    const uint64_t tsize = 1ull << tbits;
    if ((rc = ensure_scratch(g, q, std::max<uint64_t>(q->min_buf, budget), k))) return rc;
    double *wv = nullptr, *pre = nullptr;
    uint64_t *keys = nullptr;
    uint4 *wts = nullptr;
    unsigned long long *table = nullptr;
    uint32_t *ddump = nullptr;
    struct Guard {
        std::vector<void *> p;
        hipStream_t s;
        ~Guard() {
            (void)hipStreamSynchronize(s);
            for (void *x : p) dev_free(nullptr, x, 0);
        }
    } guard{{}, s};
    auto get = [&](void **ptr, uint64_t bytes) {
        int r = dev_alloc(nullptr, ptr, bytes);
        if (!r) guard.p.push_back(*ptr);
        return r;
    };
    if ((rc = get((void **)&wv, items * 8 + 8)) || (rc = get((void **)&pre, items * 8 + 8)) ||
        (rc = get((void **)&keys, budget * 8)) || (rc = get((void **)&wts, budget * 16)) ||
        (rc = get((void **)&table, tsize * 8)) || (draws && (rc = get((void **)&ddump, budget * 16))))
        return rc;
    if (scheme == TT_SAMPLE_WEDGE) k_wedge_vw<<<grid_of(items), 256, 0, s>>>(g->srstart, g->srowp, g->n, wv);
    else k_path_ew<<<grid_of((uint64_t)g->n * 64), 256, 0, s>>>(g->srstart, g->scol, g->sw, g->srowp, g->n, qexp, wv);
    HIP_TRY(hipGetLastError());
    if ((rc = inclusive_scan_f64(wv, pre, items, s, nullptr))) return rc;
    double Z = 0.0;
    HIP_TRY(hipMemcpyAsync(&Z, pre + items - 1, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!(Z > 0.0)) { // no wedge (or path) to draw: no triangle can be found
        if (draws) std::memset(draws, 0xFF, budget * 16);
        set_error("");
        return TT_OK;
    }
    const SymArgs A{g->srstart, g->scol, g->sw, g->srowp, g->n, qexp};
    const unsigned dgrid = grid_of(budget);
    if (scheme == TT_SAMPLE_WEDGE) k_wedge_draw<<<dgrid, 256, 0, s>>>(A, pre, budget, seed, keys, wts, ddump);
    else k_path_draw<<<dgrid, 256, 0, s>>>(A, pre, N, budget, seed, keys, wts, ddump);
    k_fill_u64<<<grid_of(tsize), 256, 0, s>>>(table, tsize, EMPTY_KEY);
    HIP_TRY(hipMemsetAsync(q->dcount, 0, 16, s));
    const int mode = mode_of(p);
    k_tri_distinct<<<dgrid, 256, 0, s>>>(keys, wts, budget, table, tsize - 1, mode, p, q->buf0, q->dcount);
    HIP_TRY(hipGetLastError());
    unsigned long long cnt[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(cnt, q->dcount, 16, hipMemcpyDeviceToHost, s));
    if (draws) HIP_TRY(hipMemcpyAsync(draws, ddump, budget * 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint64_t distinct = cnt[0];
    if (k && (rc = finish_topk(q, distinct, k, mode, out, n_out))) return rc;
    if (stats) {
        stats->closed_draws = cnt[1];
        stats->distinct_triangles = distinct;
    }
    set_error("");
    return TT_OK;
}
