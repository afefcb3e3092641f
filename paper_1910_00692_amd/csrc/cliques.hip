// cliques.hip — weighted edge sampling extended to 4- and 5-cliques (Sec. 4.5; Appendix A):
// edges are drawn as in Alg. 3, and every clique of the requested size that contains a drawn
// edge is enumerated; the answer is the top-k of those cliques by the generalized p-mean of
// their C(s, 2) edge weights (Eq. 1 over the clique's edges).
//
// One wave per drawn edge {u, v}: the common neighbours C of u and v (the lanes split u's row
// of the symmetric adjacency and search v's) are kept in LDS with their two weights; then the
// lanes split the pairs (4-cliques) or pairs-then-thirds (5-cliques) of C and look the
// remaining edges up in the symmetric rows.  A clique holding several drawn edges is reported
// once, from the drawn edge of smallest oriented-entry position.
//
// Order key (one 64-bit word): the sum of the weights at p = 1, the max / min at p = +-inf, the
// FP64 bits of the mean otherwise; ties by the sorted vertex IDs.  A record reuses the triangle
// record (key, then the first two IDs complemented so that smaller IDs rank first, then the
// last three), so the triangle selection sorts cliques too.
#include <cmath>
#include <cstring>

#include "common.h"
#include "enum.h"

namespace {

constexpr uint32_t CQ_MAX = 512; // common neighbours a wave keeps (more: the call reports it)

struct CliqueArgs {
    const uint64_t *srstart;
    const uint32_t *scol, *sw;
    const uint64_t *rstart;
    const uint32_t *rlen, *col, *deg;
    const uint8_t *emark;
    const uint32_t *mlist; // drawn entries (head-sorted positions)
    uint64_t nmarked;
    const uint32_t *osrc, *ocol, *owgt;
    uint32_t size;
    int mode;
    double p;
    trec *out;
    unsigned long long *count; // [0] records, [1] waves whose common neighbours overflowed
    uint64_t cap;
};

__device__ __forceinline__ uint64_t srow_find(const CliqueArgs &A, uint32_t a, uint32_t b, uint32_t *w) {
    uint64_t lo = A.srstart[a], hi = A.srstart[a + 1];
    const uint64_t end = hi;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (A.scol[mid] < b) lo = mid + 1; else hi = mid;
    }
    if (lo < end && A.scol[lo] == b) {
        *w = A.sw[lo];
        return lo;
    }
    return ~0ull;
}

// Head-sorted position of the oriented entry of edge {a, b} (tail: lower in (degree, ID)).
__device__ __forceinline__ uint64_t entry_of(const CliqueArgs &A, uint32_t a, uint32_t b) {
    const uint32_t da = A.deg[a], db = A.deg[b];
    if (da > db || (da == db && a > b)) { const uint32_t t = a; a = b; b = t; }
    uint64_t lo = A.rstart[a], hi = lo + A.rlen[a];
    const uint64_t end = hi;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (A.col[mid] < b) lo = mid + 1; else hi = mid;
    }
    return lo < end && A.col[lo] == b ? lo : ~0ull;
}

// True if no other edge of the clique is drawn at a smaller entry position than `me`.
__device__ __forceinline__ bool reported_here(const CliqueArgs &A, const uint32_t *v, uint32_t s, uint64_t me) {
    for (uint32_t x = 0; x < s; x++)
        for (uint32_t y = x + 1; y < s; y++) {
            const uint64_t e = entry_of(A, v[x], v[y]);
            if (e < me && A.emark[e]) return false;
        }
    return true;
}

// The clique's order key from its E = s (s - 1) / 2 weights.
__device__ uint64_t clique_key(int mode, double p, const uint32_t *w, uint32_t E) {
    if (mode == MODE_MAX || mode == MODE_MIN) {
        uint32_t r = w[0];
        for (uint32_t t = 1; t < E; t++) r = mode == MODE_MAX ? (w[t] > r ? w[t] : r) : (w[t] < r ? w[t] : r);
        return r;
    }
    if (mode == MODE_SUM) {
        uint64_t r = 0;
        for (uint32_t t = 0; t < E; t++) r += w[t];
        return r;
    }
    double m;
    if (mode == MODE_PROD) { // geometric mean
        double acc = 0.0;
        for (uint32_t t = 0; t < E; t++) acc += log((double)w[t]);
        m = exp(acc / (double)E);
    } else { // m = s exp(log1p(mean(expm1(p log(x / s)))) / p), s = max (p > 0) or min (p < 0)
        double sref = (double)w[0];
        for (uint32_t t = 1; t < E; t++) sref = p > 0 ? fmax(sref, (double)w[t]) : fmin(sref, (double)w[t]);
        double acc = 0.0;
        for (uint32_t t = 0; t < E; t++) acc += expm1(p * log((double)w[t] / sref));
        m = sref * exp(log1p(acc / (double)E) / p);
    }
    return __builtin_bit_cast(uint64_t, m);
}

__device__ __forceinline__ void emit(const CliqueArgs &A, const uint32_t *vin, const uint32_t *w, uint32_t s) {
    uint32_t v[5];
    for (uint32_t t = 0; t < s; t++) v[t] = vin[t];
    for (uint32_t a = 1; a < s; a++) // insertion sort of at most 5 IDs
        for (uint32_t b = a; b > 0 && v[b - 1] > v[b]; b--) { const uint32_t x = v[b]; v[b] = v[b - 1]; v[b - 1] = x; }
    trec r;
    r.khi = clique_key(A.mode, A.p, w, s * (s - 1) / 2);
    r.klo = ~(((uint64_t)v[0] << 32) | v[1]);
    r.i = v[2];
    r.j = v[3];
    r.l = s == 5 ? v[4] : 0u;
    r.pad = 0;
    const unsigned long long slot = atomicAdd(&A.count[0], 1ull);
    if (slot < A.cap) A.out[slot] = r;
}

// Pair index -> (x, y), x < y < c, over the pairs listed row by row.
__device__ __forceinline__ void pair_of(uint64_t idx, uint32_t c, uint32_t &x, uint32_t &y) {
    // x is the largest with x (2c - x - 1) / 2 <= idx
    double cc = (double)c;
    uint32_t t = (uint32_t)floor((2.0 * cc - 1.0 - sqrt((2.0 * cc - 1.0) * (2.0 * cc - 1.0) - 8.0 * (double)idx)) / 2.0);
    while (t > 0 && (uint64_t)t * (2 * c - t - 1) / 2 > idx) t--;
    while ((uint64_t)(t + 1) * (2 * c - t - 2) / 2 <= idx) t++;
    x = t;
    y = (uint32_t)(idx - (uint64_t)t * (2 * c - t - 1) / 2) + t + 1;
}

__global__ __launch_bounds__(256) void k_cliques(CliqueArgs A) {
    __shared__ uint32_t cv[4][CQ_MAX], cwu[4][CQ_MAX], cwv[4][CQ_MAX];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t t = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; t < A.nmarked; t += nw) {
        const uint64_t me = A.mlist[t];
        const uint32_t u = A.osrc[me], v = A.ocol[me], wuv = A.owgt[me];
        // common neighbours: u's row split over the lanes, each searched in v's row; the wave's
        // slots in LDS are handed out by a wave-uniform running count
        uint32_t nc = 0;
        const uint64_t lo = A.srstart[u], hi = A.srstart[u + 1];
        __builtin_amdgcn_wave_barrier(); // the previous edge's reads of the slots come first
        for (uint64_t b = lo; b < hi; b += 64) {
            uint32_t c = 0, wu = 0, wvv = 0;
            bool hit = false;
            if (b + lane < hi) {
                c = A.scol[b + lane];
                wu = A.sw[b + lane];
                hit = c != v && srow_find(A, v, c, &wvv) != ~0ull;
            }
            const uint64_t bal = __ballot(hit);
            const uint32_t r = nc + __popcll(bal & ((1ull << lane) - 1ull));
            if (hit && r < CQ_MAX) {
                cv[wv][r] = c;
                cwu[wv][r] = wu;
                cwv[wv][r] = wvv;
            }
            nc += __popcll(bal);
        }
        __threadfence_block();
        __builtin_amdgcn_wave_barrier(); // the slots are written before any lane reads them
        if (nc > CQ_MAX) {
            if (lane == 0) atomicAdd(&A.count[1], 1ull);
            continue;
        }
        const uint64_t pairs = (uint64_t)nc * (nc - 1) / 2;
        for (uint64_t idx = lane; idx < pairs; idx += 64) {
            uint32_t x, y;
            pair_of(idx, nc, x, y);
            uint32_t wxy;
            if (srow_find(A, cv[wv][x], cv[wv][y], &wxy) == ~0ull) continue;
            if (A.size == 4) {
                const uint32_t vs[4] = {u, v, cv[wv][x], cv[wv][y]};
                const uint32_t ws[6] = {wuv, cwu[wv][x], cwu[wv][y], cwv[wv][x], cwv[wv][y], wxy};
                if (reported_here(A, vs, 4, me)) emit(A, vs, ws, 4);
            } else {
                for (uint32_t z = y + 1; z < nc; z++) {
                    uint32_t wxz, wyz;
                    if (srow_find(A, cv[wv][x], cv[wv][z], &wxz) == ~0ull) continue;
                    if (srow_find(A, cv[wv][y], cv[wv][z], &wyz) == ~0ull) continue;
                    const uint32_t vs[5] = {u, v, cv[wv][x], cv[wv][y], cv[wv][z]};
                    const uint32_t ws[10] = {wuv, cwu[wv][x], cwu[wv][y], cwu[wv][z], cwv[wv][x],
                                             cwv[wv][y], cwv[wv][z], wxy, wxz, wyz};
                    if (reported_here(A, vs, 5, me)) emit(A, vs, ws, 5);
                }
            }
        }
    }
}

// Positions of the drawn entries (or of every entry), compacted.
__global__ __launch_bounds__(256) void k_list_marked(const uint8_t *emark, uint64_t m, bool all, uint32_t *list,
                                                     unsigned long long *count) {
    const int lane = threadIdx.x & 63;
    for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~63ull; base < m;
         base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = base + lane;
        const bool keep = e < m && (all || emark[e]);
        const uint64_t bal = __ballot(keep);
        if (!bal) continue;
        unsigned long long b0 = 0;
        if (lane == 0) b0 = atomicAdd(count, (unsigned long long)__popcll(bal));
        b0 = __shfl(b0, 0, 64);
        if (keep) list[b0 + __popcll(bal & ((1ull << lane) - 1ull))] = (uint32_t)e;
    }
}

__global__ void k_clique_out(const trec *in, uint32_t K, uint32_t s, int mode, tt_clique *out) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K) return;
    const trec r = in[t];
    const uint64_t ids = ~r.klo;
    tt_clique o;
    o.v[0] = (uint32_t)(ids >> 32);
    o.v[1] = (uint32_t)ids;
    o.v[2] = r.i;
    o.v[3] = r.j;
    o.v[4] = s == 5 ? r.l : 0u;
    o.size = s;
    const double E = (double)(s * (s - 1) / 2);
    if (mode == MODE_MAX || mode == MODE_MIN) o.score = (double)r.khi;
    else if (mode == MODE_SUM) o.score = (double)r.khi / E;
    else o.score = __builtin_bit_cast(double, r.khi);
    out[t] = o;
}

unsigned grid_of(uint64_t items) {
    const uint64_t b = (items + 255) / 256, cap = (uint64_t)num_cus() * 16;
    return (unsigned)std::max<uint64_t>(1, std::min(b, cap));
}

} // namespace

extern "C" int sample_heavy_cliques(tt_graph *g, uint32_t size, uint32_t k, double p, uint64_t budget, uint64_t seed,
                                    double qexp, uint32_t flags, tt_clique *out, uint32_t *n_out, uint64_t *found) {
    if (n_out) *n_out = 0;
    if (found) *found = 0;
    if (!g || !n_out) return fail(TT_E_ARG, "graph or n_out is NULL");
    if (size != 4 && size != 5) return fail(TT_E_ARG, "clique size must be 4 or 5");
    if (std::isnan(p)) return fail(TT_E_ARG, "p is NaN");
    if (k && !out) return fail(TT_E_ARG, "out is NULL");
    if (!std::isnan(qexp) && !(qexp > 0.0 && std::isfinite(qexp)))
        return fail(TT_E_ARG, "the sampling exponent q must be finite and > 0 (or NaN for the default)");
    const bool all = (flags & TT_CLIQUE_ALL_EDGES) != 0;
    if (k == 0 || g->m == 0 || (budget == 0 && !all)) { set_error(""); return TT_OK; }
    if (std::isnan(qexp)) qexp = (std::isfinite(p) && p > 0.0) ? p : 1.0;
    std::lock_guard<std::mutex> lock(g->mu);
    (void)hipSetDevice(g->device);
    QueryCtx *q = &g->q;
    hipStream_t s = q->stream;
    int rc;
    if ((rc = ensure_sym(g, s))) return rc;
    if ((rc = ensure_scratch(g, q, std::max<uint64_t>(q->min_buf, 16ull * k), k))) return rc;
    if (!all && (rc = es_mark_edges(g, q, qexp, budget, seed))) return rc;
    uint32_t *mlist = nullptr;
    tt_clique *dout = nullptr;
    struct Guard {
        void *a, *b;
        hipStream_t s;
        ~Guard() {
            (void)hipStreamSynchronize(s);
            dev_free(nullptr, a, 0);
            dev_free(nullptr, b, 0);
        }
    } guard{nullptr, nullptr, s};
    if ((rc = dev_alloc(nullptr, (void **)&mlist, g->m * 4 + 4))) return rc;
    guard.a = mlist;
    if ((rc = dev_alloc(nullptr, (void **)&dout, (uint64_t)k * sizeof(tt_clique)))) return rc;
    guard.b = dout;
    HIP_TRY(hipMemsetAsync(q->dcount, 0, 4 * sizeof(unsigned long long), s));
    k_list_marked<<<grid_of(g->m), 256, 0, s>>>(g->emark, g->m, all, mlist, q->dcount + 2);
    HIP_TRY(hipGetLastError());
    unsigned long long nm = 0;
    HIP_TRY(hipMemcpyAsync(&nm, q->dcount + 2, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int mode = mode_of(p) == MODE_SUMSQ ? MODE_GEN : mode_of(p); // p = 2: FP64 like any other p
    CliqueArgs A;
    A.srstart = g->srstart;
    A.scol = g->scol;
    A.sw = g->sw;
    A.rstart = g->rstart;
    A.rlen = g->rlen;
    A.col = g->col;
    A.deg = g->deg;
    A.emark = all ? nullptr : g->emark;
    A.mlist = mlist;
    A.nmarked = nm;
    A.osrc = g->osrc;
    A.ocol = g->col;
    A.owgt = g->wgt;
    A.size = size;
    A.mode = mode;
    A.p = p;
    A.out = q->buf0;
    A.count = q->dcount;
    A.cap = q->buf_cap;
    if (all) {
        // every edge drawn: a clique is reported from its entry of smallest position, which
        // reported_here checks through the marks; give it an all-ones mark array
        if (!g->emark && (rc = dev_alloc(g, (void **)&g->emark, g->m + 1))) return rc;
        HIP_TRY(hipMemsetAsync(g->emark, 1, g->m + 1, s));
        A.emark = g->emark;
    }
    if (nm) k_cliques<<<grid_of(nm * 64), 256, 0, s>>>(A);
    HIP_TRY(hipGetLastError());
    unsigned long long cnt[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(cnt, q->dcount, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (cnt[1]) return fail(TT_E_TOO_LARGE, "a drawn edge has more than 512 common neighbours");
    if (cnt[0] > q->buf_cap) return fail(TT_E_TOO_LARGE, "more cliques on the drawn edges than the buffer holds");
    if (found) *found = cnt[0];
    const uint32_t K = (uint32_t)std::min<uint64_t>(cnt[0], k);
    if (K) {
        trec *res = nullptr; // selected with the triangle records' order, then written as cliques
        if ((rc = select_records(q, cnt[0], k, &res))) return rc;
        k_clique_out<<<(K + 255) / 256, 256, 0, s>>>(res, K, size, mode, dout);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(out, dout, (size_t)K * sizeof(tt_clique), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    *n_out = K;
    set_error("");
    return TT_OK;
}
