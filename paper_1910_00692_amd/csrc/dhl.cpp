// dhl.cpp — the paper's own exact method on the CPU: the dynamic heavy-light algorithm
// (Alg. 2, Sec. 3.1) with a fixed pointer exponent alpha_p (Eq. ptr_values), and its
// distribution-oblivious variant Auto-HL (Sec. 3.3), which picks the pointer to advance from
// running estimates of the threshold's rate of decrease per unit of work.
//
// The edges are sorted by weight (descending; ties by input index) and split by two pointers
// h <= l into super-heavy S = ranks [0, h], heavy H = (h, l] and light L = (l, m).  Advancing l
// moves the edge of rank l+1 from L to H and enumerates its triangles with one edge in H and
// one in L (its triangles with an edge in S, or with both others in S u H, were enumerated
// earlier); advancing h moves the edge of rank h+1 from H to S and enumerates its triangles
// whose two other edges are in L.  Each triangle is therefore enumerated exactly once, and
// after every step all triangles with an edge in S or two edges in S u H are known.  A
// triangle not yet enumerated has no edge in S and at most one in H, so its p-mean is at most
// m_p(w_{h+1}, w_{l+1}, w_{l+2}) (m_p is non-decreasing in each weight, for every p); the
// algorithm stops once k known triangles rank strictly above that bound.
//
// The pointer rule: the printed condition compares w_{l+1} with w_{h+1}^alpha, while the
// analysis keeps w_h ~ w_l^alpha (alpha_p = 2 - p / (p - 1 + beta) > 1); this code follows the
// analysis and advances l while w_{l+1}^alpha >= w_{h+1} (and whenever H is empty).
//
// Host code only (g++, OpenMP for the sort and the adjacency build).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <queue>
#include <string>
#include <vector>

#include <omp.h>

#include "../../include/topktri_dhl.h"

namespace {

typedef unsigned __int128 u128;
enum { K_MAX = 0, K_MIN = 1, K_SUM = 2, K_SUMSQ = 3, K_PROD = 4, K_GEN = 5 };

thread_local std::string last_error;
int fail(int code, const char *msg) {
    last_error = msg;
    return code;
}

int kind_of(double p) {
    if (std::isinf(p)) return p > 0 ? K_MAX : K_MIN;
    if (p == 1.0) return K_SUM;
    if (p == 2.0) return K_SUMSQ;
    if (p == 0.0) return K_PROD;
    return K_GEN;
}

// Eq. 1 for a generic p without overflow: m = s exp(log1p(mean(expm1(p log(x/s)))) / p), with
// s the largest weight for p > 0 and the smallest for p < 0.
double gen_mean(double p, double a, double b, double c) {
    const double s = p > 0 ? std::max(a, std::max(b, c)) : std::min(a, std::min(b, c));
    const double t = std::expm1(p * std::log(a / s)) + std::expm1(p * std::log(b / s)) + std::expm1(p * std::log(c / s));
    return s * std::exp(std::log1p(t / 3.0) / p);
}

// A key that orders triangles like m_p: exact integers for the means named after Eq. 1 (and
// p = 2), the FP64 bits of m_p otherwise (positive doubles order like their bits).
u128 key_of(int kind, double p, uint32_t a, uint32_t b, uint32_t c) {
    switch (kind) {
    case K_MAX: return std::max(a, std::max(b, c));
    case K_MIN: return std::min(a, std::min(b, c));
    case K_SUM: return (u128)a + b + c;
    case K_SUMSQ: return (u128)a * a + (u128)b * b + (u128)c * c;
    case K_PROD: return (u128)a * b * c;
    default: {
        const double m = gen_mean(p, a, b, c);
        uint64_t bits;
        std::memcpy(&bits, &m, 8);
        return bits;
    }
    }
}

double score_of(int kind, u128 key) {
    switch (kind) {
    case K_MAX:
    case K_MIN: return (double)(uint64_t)key;
    case K_SUM: return (double)(uint64_t)key / 3.0;
    case K_SUMSQ: return std::sqrt((double)key / 3.0);
    case K_PROD: return std::cbrt((double)key);
    default: {
        double d;
        const uint64_t bits = (uint64_t)key;
        std::memcpy(&d, &bits, 8);
        return d;
    }
    }
}

struct Rec {
    u128 key;
    uint32_t i, j, l;
};
// a ranks before b: larger key, then smaller (i, j, l)
bool better(const Rec &a, const Rec &b) {
    if (a.key != b.key) return a.key > b.key;
    if (a.i != b.i) return a.i < b.i;
    if (a.j != b.j) return a.j < b.j;
    return a.l < b.l;
}
struct WorstOnTop {
    bool operator()(const Rec &a, const Rec &b) const { return better(a, b); }
};

struct Graph {
    uint32_t n = 0;
    uint64_t m = 0;
    std::vector<uint32_t> order;  // edge ids by (weight desc, id)
    std::vector<uint32_t> ws;     // ws[r] = weight of the edge of rank r
    std::vector<uint32_t> ea, eb; // ends of the edge of rank r
    // symmetric adjacency, rows sorted by neighbour: neighbour and edge rank
    std::vector<uint64_t> rp;
    std::vector<uint32_t> nb, nr;
    // the same rows sorted by edge rank: the S u H entries of a row are a prefix
    std::vector<uint32_t> rnb, rnr;
};

// Validation (vertex range, self-loop, zero weight, duplicate pair: the first failing rule of
// the simple-graph, positive-weight requirement), sort, adjacency.
int build(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w, Graph &G,
          double &sort_ms) {
    bool range = false, loop = false, zero = false;
#pragma omp parallel for reduction(|| : range, loop, zero) schedule(static)
    for (int64_t e = 0; e < (int64_t)m; e++) {
        if (src[e] >= n || dst[e] >= n) range = true;
        else if (src[e] == dst[e]) loop = true;
        if (w[e] == 0) zero = true;
    }
    if (range) return fail(TT_E_VERTEX_RANGE, "an endpoint >= n");
    if (loop) return fail(TT_E_SELF_LOOP, "a self-loop");
    if (zero) return fail(TT_E_ZERO_WEIGHT, "a zero weight");
    G.n = n;
    G.m = m;
    const auto t0 = std::chrono::steady_clock::now();
    G.order.resize(m);
    for (uint64_t e = 0; e < m; e++) G.order[e] = (uint32_t)e;
    // parallel sort: each thread sorts a block, then pairwise merges
    auto cmp = [&](uint32_t x, uint32_t y) { return w[x] != w[y] ? w[x] > w[y] : x < y; };
    {
        const int T = omp_get_max_threads();
        std::vector<uint64_t> cut(T + 1);
        for (int t = 0; t <= T; t++) cut[t] = m * t / T;
#pragma omp parallel for schedule(static, 1)
        for (int t = 0; t < T; t++) std::sort(G.order.begin() + cut[t], G.order.begin() + cut[t + 1], cmp);
        for (int width = 1; width < T; width *= 2) {
#pragma omp parallel for schedule(dynamic, 1)
            for (int t = 0; t < T; t += 2 * width) {
                const int mid = std::min(t + width, T), hi = std::min(t + 2 * width, T);
                std::inplace_merge(G.order.begin() + cut[t], G.order.begin() + cut[mid], G.order.begin() + cut[hi], cmp);
            }
        }
    }
    sort_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    G.ws.resize(m);
    G.ea.resize(m);
    G.eb.resize(m);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < (int64_t)m; r++) {
        const uint32_t e = G.order[r];
        G.ws[r] = w[e];
        G.ea[r] = src[e];
        G.eb[r] = dst[e];
    }
    G.rp.assign((uint64_t)n + 1, 0);
    for (uint64_t e = 0; e < m; e++) {
        G.rp[src[e] + 1]++;
        G.rp[dst[e] + 1]++;
    }
    for (uint64_t v = 0; v < n; v++) G.rp[v + 1] += G.rp[v];
    G.nb.resize(2 * m);
    G.nr.resize(2 * m);
    G.rnb.resize(2 * m);
    G.rnr.resize(2 * m);
    {
        std::vector<uint64_t> cur(G.rp.begin(), G.rp.end() - 1);
        // by rank: the rank-sorted rows come out in order
        for (uint64_t r = 0; r < m; r++) {
            const uint32_t a = G.ea[r], b = G.eb[r];
            uint64_t x = cur[a]++, y = cur[b]++;
            G.rnb[x] = b; G.rnr[x] = (uint32_t)r;
            G.rnb[y] = a; G.rnr[y] = (uint32_t)r;
        }
    }
    bool dup = false;
#pragma omp parallel reduction(|| : dup)
    {
        std::vector<std::pair<uint32_t, uint32_t>> tmp;
#pragma omp for schedule(dynamic, 1024)
        for (int64_t v = 0; v < (int64_t)n; v++) {
            const uint64_t lo = G.rp[v], hi = G.rp[v + 1];
            tmp.clear();
            for (uint64_t t = lo; t < hi; t++) tmp.push_back({G.rnb[t], G.rnr[t]});
            std::sort(tmp.begin(), tmp.end());
            for (uint64_t t = lo; t < hi; t++) {
                G.nb[t] = tmp[t - lo].first;
                G.nr[t] = tmp[t - lo].second;
                if (t > lo && G.nb[t] == G.nb[t - 1]) dup = true;
            }
        }
    }
    if (dup) return fail(TT_E_DUP_EDGE, "the same unordered pair twice");
    return TT_OK;
}

// rank of edge (v, c), or UINT32_MAX if there is none
inline uint32_t rank_of(const Graph &G, uint32_t v, uint32_t c) {
    uint64_t lo = G.rp[v], hi = G.rp[v + 1];
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (G.nb[mid] < c) lo = mid + 1; else hi = mid;
    }
    return lo < G.rp[v + 1] && G.nb[lo] == c ? G.nr[lo] : UINT32_MAX;
}

struct Run {
    const Graph &G;
    int kind;
    double p;
    uint32_t k;
    std::priority_queue<Rec, std::vector<Rec>, WorstOnTop> heap;
    uint64_t found = 0;
    Run(const Graph &g, int kd, double pp, uint32_t kk) : G(g), kind(kd), p(pp), k(kk) {}

    void add(uint32_t a, uint32_t b, uint32_t c, uint32_t wab, uint32_t wac, uint32_t wbc) {
        found++;
        Rec r;
        r.key = key_of(kind, p, wab, wac, wbc);
        uint32_t x = a, y = b, z = c, t;
        if (x > y) { t = x; x = y; y = t; }
        if (y > z) { t = y; y = z; z = t; }
        if (x > y) { t = x; x = y; y = t; }
        r.i = x; r.j = y; r.l = z;
        if (heap.size() < k) heap.push(r);
        else if (better(r, heap.top())) { heap.pop(); heap.push(r); }
    }
};

} // namespace

extern "C" const char *dhl_last_error(void) { return last_error.c_str(); }

extern "C" int dhl_topk_triangles(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                                  uint32_t k, double p, double alpha, int threads, tt_triangle *out, uint32_t *n_out,
                                  tt_dhl_stats *stats) {
    if (n_out) *n_out = 0;
    if (!n_out || (m && (!src || !dst || !w)) || (k && !out) || std::isnan(p))
        return fail(TT_E_ARG, "NULL argument or NaN p");
    if (!(alpha >= 0.0) || std::isinf(alpha)) return fail(TT_E_ARG, "alpha must be >= 0 (0: Auto-HL) and finite");
    if (m > 0xFFFFFFFEull || n > 0xFFFFFFFEu) return fail(TT_E_TOO_LARGE, "n and m must be < 2^32 - 1");
    if (threads > 0) omp_set_num_threads(threads);
    const auto t0 = std::chrono::steady_clock::now();
    tt_dhl_stats st;
    std::memset(&st, 0, sizeof(st));
    Graph G;
    int rc = build(n, m, src, dst, w, G, st.sort_ms);
    if (rc) return rc;
    const auto t1 = std::chrono::steady_clock::now();
    st.build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (k == 0 || m < 3) {
        if (stats) *stats = st;
        last_error.clear();
        return TT_OK;
    }
    const int kind = kind_of(p);
    Run R(G, kind, p, k);
    std::vector<uint32_t> hcnt(n, 0), scnt(n, 0); // per vertex: entries of rank <= l, <= h
    int64_t h = -1, l = -1;
    const bool automatic = alpha == 0.0;
    // Auto-HL: weight step per edge at a rank (the gap to the next smaller weight, spread over
    // the edges of that weight), from the sorted weights
    auto step_at = [&](uint64_t r) -> double {
        const uint32_t wr = G.ws[r];
        uint64_t lo = r, hi = r;
        // edges of this weight: a run around r (bounded scan, then binary search)
        {
            uint64_t a = 0, b = r;
            while (a < b) { const uint64_t mid = (a + b) >> 1; if (G.ws[mid] > wr) a = mid + 1; else b = mid; }
            lo = a;
            a = r; b = G.m;
            while (a < b) { const uint64_t mid = (a + b) >> 1; if (G.ws[mid] >= wr) a = mid + 1; else b = mid; }
            hi = a;
        }
        const double next = hi < G.m ? (double)G.ws[hi] : 0.0;
        return ((double)wr - next) / (double)(hi - lo);
    };
    auto pw = [&](double x) { return (kind == K_GEN || kind == K_SUMSQ) ? std::pow(x, p - 1.0) : 1.0; };
    const double slack = kind == K_GEN ? 1e-12 : 0.0;
    for (;;) {
        if (l + 2 >= (int64_t)G.m) break; // fewer than two light edges: every triangle is known
        const u128 bound = key_of(kind, p, G.ws[h + 1], G.ws[l + 1], G.ws[l + 2]);
        if (R.heap.size() == k) {
            const Rec &kth = R.heap.top();
            bool above = kth.key > bound;
            if (above && kind == K_GEN) {
                double a, b;
                const uint64_t ka = (uint64_t)kth.key, kb = (uint64_t)bound;
                std::memcpy(&a, &ka, 8);
                std::memcpy(&b, &kb, 8);
                above = a > b * (1.0 + slack);
            }
            if (above) break;
        }
        bool move_l;
        if (h + 1 > l) move_l = true; // H is empty
        else if (!automatic) move_l = std::pow((double)G.ws[l + 1], alpha) >= (double)G.ws[h + 1];
        else {
            // Eq. ptr_values: advance the pointer with the larger w^(p-1) dw/dt, where dw is the
            // weight step per edge and dt the work of the move (degrees of the moving edge's
            // ends in G[L] for h, in G[S u H] for l)
            const uint64_t rh = (uint64_t)(h + 1), rl = (uint64_t)(l + 1);
            const uint32_t ha = G.ea[rh], hb = G.eb[rh], la = G.ea[rl], lb = G.eb[rl];
            const double cost_h = 1.0 + (double)(G.rp[ha + 1] - G.rp[ha] - hcnt[ha]) + (double)(G.rp[hb + 1] - G.rp[hb] - hcnt[hb]);
            const double cost_l = 1.0 + (double)(hcnt[la] - scnt[la]) + (double)(hcnt[lb] - scnt[lb]);
            const double gain_h = pw(G.ws[rh]) * step_at(rh) / cost_h;
            const double gain_l = 2.0 * pw(G.ws[rl]) * step_at(rl) / cost_l;
            move_l = gain_l >= gain_h;
        }
        if (move_l) {
            const uint32_t r = (uint32_t)(l + 1), a = G.ea[r], b = G.eb[r], wab = G.ws[r];
            // triangles of edge r with one other edge in H (rank in (h, l]) and the last in L
            for (int side = 0; side < 2; side++) {
                const uint32_t x = side ? b : a, y = side ? a : b;
                for (uint64_t t = G.rp[x] + scnt[x]; t < G.rp[x] + hcnt[x]; t++) {
                    const uint32_t c = G.rnb[t], rxc = G.rnr[t];
                    const uint32_t ryc = rank_of(G, y, c);
                    if (ryc == UINT32_MAX || ryc <= r) continue;
                    if (side == 0) R.add(a, b, c, wab, G.ws[rxc], G.ws[ryc]);
                    else R.add(a, b, c, wab, G.ws[ryc], G.ws[rxc]);
                }
                st.lookups += hcnt[x] - scnt[x];
            }
            hcnt[a]++;
            hcnt[b]++;
            l = r;
            st.l_moves++;
        } else {
            const uint32_t r = (uint32_t)(h + 1), a = G.ea[r], b = G.eb[r], wab = G.ws[r];
            // triangles of edge r whose two other edges are in L (rank > l): the shorter row is
            // scanned, each neighbour looked up in the other row
            const bool a_short = G.rp[a + 1] - G.rp[a] <= G.rp[b + 1] - G.rp[b];
            const uint32_t x = a_short ? a : b, y = a_short ? b : a;
            for (uint64_t t = G.rp[x]; t < G.rp[x + 1]; t++) {
                const uint32_t rxc = G.nr[t];
                if ((int64_t)rxc <= l) continue;
                const uint32_t c = G.nb[t];
                const uint32_t ryc = rank_of(G, y, c);
                if (ryc == UINT32_MAX || (int64_t)ryc <= l) continue;
                if (a_short) R.add(a, b, c, wab, G.ws[rxc], G.ws[ryc]);
                else R.add(a, b, c, wab, G.ws[ryc], G.ws[rxc]);
            }
            st.lookups += G.rp[x + 1] - G.rp[x];
            scnt[a]++;
            scnt[b]++;
            h = r;
            st.h_moves++;
        }
    }
    std::vector<Rec> res;
    res.reserve(R.heap.size());
    while (!R.heap.empty()) {
        res.push_back(R.heap.top());
        R.heap.pop();
    }
    std::sort(res.begin(), res.end(), better);
    for (size_t t = 0; t < res.size(); t++) {
        out[t].i = res[t].i;
        out[t].j = res[t].j;
        out[t].l = res[t].l;
        out[t]._pad = 0;
        out[t].score = score_of(kind, res[t].key);
    }
    *n_out = (uint32_t)res.size();
    st.enumerated = R.found;
    st.final_h = (uint64_t)(h + 1);
    st.final_l = (uint64_t)(l + 1);
    const auto t2 = std::chrono::steady_clock::now();
    st.loop_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
    st.total_ms = std::chrono::duration<double, std::milli>(t2 - t0).count();
    if (stats) *stats = st;
    last_error.clear();
    return TT_OK;
}
