// common.h — internal declarations shared by the library's translation units.
//
// Nothing here is part of the public ABI (include/topktri.h is).  All device code targets
// gfx950: 64-lane wavefronts, no MFMA (the work is integer graph traversal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>
#include <mutex>
#include <atomic>
#include <algorithm>
#include <new>

#include "../../include/topktri.h"

typedef unsigned __int128 u128;

// ----------------------------------------------------------------------------- scoring modes
// The order of triangles under Eq. 1 is decided by a key that is a monotone transform of
// m_p: exact integers for the means named after Eq. 1 (and p = 2), FP64 bits otherwise.
enum { MODE_MAX = 0, MODE_MIN = 1, MODE_SUM = 2, MODE_SUMSQ = 3, MODE_PROD = 4, MODE_GEN = 5 };

inline int mode_of(double p) {
    if (p == __builtin_inf()) return MODE_MAX;
    if (p == -__builtin_inf()) return MODE_MIN;
    if (p == 1.0) return MODE_SUM;
    if (p == 2.0) return MODE_SUMSQ;
    if (p == 0.0) return MODE_PROD;
    return MODE_GEN;
}

// One candidate triangle in device memory: order key (hi, lo) and original IDs i < j < l.
struct __attribute__((aligned(16))) trec {
    uint64_t khi, klo;
    uint32_t i, j, l, pad;
};

// A candidate base entry u->v of the current pass: tail, head, weight, head-sorted position.
struct cand {
    uint32_t u, v, a, pos;
};

// A candidate with many entries to intersect, handed from the wave that found it to a kernel
// that spreads its entries over many waves (56 bytes).
struct Heavy {
    uint64_t Ab, Bb;           // iterated row (weight-sorted copy), other row (both copies)
    uint32_t qA, qB, Blen, zB; // admissible entries of each row, other row's length and floor
    uint32_t a, u, v, fl;      // base entry weight and ends, filter flags
    uint32_t g, pad;           // graph (batched form)
};
constexpr uint32_t HEAVY_CAP = 16384;    // heavy candidates per piece of a pass (more stay in-wave)
constexpr uint32_t HEAVY_PIECE = 256;    // entries of a heavy candidate's row taken by one wave
constexpr uint32_t HEAVY_PIECES = 65536; // pieces listed per piece of a pass

// ----------------------------------------------------------------------------- query state
// Device state of one query in flight: its stream, candidate buffers and counters.  A graph
// owns one for its synchronous calls; a server owns one per slot, so that queries on one
// resident graph run concurrently on separate streams.
// What an intersection needs of a vertex, in one 16-byte load.
struct alignas(16) VInfo {
    uint64_t rstart; // first entry of the out-row
    uint32_t rlen;   // out-degree
    uint32_t maxw;   // largest weight in the out-row
};

struct BoundOrder;
struct QueryCtx {
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    trec *buf0 = nullptr, *buf1 = nullptr; // triangle buffer and its sort ping-pong
    uint64_t buf_cap = 0;
    struct cand *cand = nullptr;           // candidate entries of the current piece of a pass
    uint64_t cand_cap = 0;
    uint64_t max_cand = 1ull << 27;        // a pass streams its entries in pieces of this size
    uint64_t min_buf = 1ull << 22;         // smallest triangle buffer (records)
    uint32_t *ccnt = nullptr;              // candidates per filter block
    struct Heavy *heavy = nullptr;         // [HEAVY_CAP] heavy candidates of the current piece
    unsigned long long *nheavy = nullptr;  // [0] heavy candidates, [1] pieces (reset by the filter)
    uint2 *hpiece = nullptr;               // [HEAVY_PIECES] (heavy candidate, piece number)
    unsigned long long *spart = nullptr;   // spread per-pass counters
    unsigned long long *dcount = nullptr;  // [16] counters
    unsigned long long *hcount = nullptr;  // pinned mirror
    tt_triangle *dout = nullptr;
    uint64_t dout_cap = 0;
    tt_triangle *hout = nullptr;           // pinned host staging of the results (dout_cap records)
    uint8_t *vflag = nullptr;              // [n]
    uint8_t *vflag2 = nullptr;             // [n]
    // subset queries: the entries that can be the base of a triangle touching the subset
    uint32_t *sub_src = nullptr, *sub_col = nullptr, *sub_wgt = nullptr, *sub_pos = nullptr;
    uint32_t *sub_vlist = nullptr;         // in-neighbours of the subset (outside it)
    // for each listed in-neighbour u (by its index in sub_vlist): its out-neighbours c in the
    // subset and the weights of u->c, as a run [sp_start, sp_start + sp_cnt) of sp_c / sp_w
    uint32_t *sp_c = nullptr, *sp_w = nullptr, *sp_start = nullptr, *sp_cnt = nullptr;
    uint64_t sub_cap = 1ull << 24;         // capacity of the compact stream and of the list
    uint64_t sub_len = 0;                  // entries in the compact stream
    bool sub_active = false;               // the passes stream the compact list
    std::vector<uint64_t> sub_hist;        // host: its entries per weight_bin(w)
    BoundOrder *ord = nullptr;             // bound order of the running query's p (or NULL)
    // A context whose device scratch is a fixed region handed in by the caller of the
    // no-allocation query: it allocates nothing (no device or pinned memory, no events), builds
    // nothing of the graph lazily (streams and bound orders are used only once placed), and
    // copies the results straight to the caller's buffer.
    bool fixed = false;
    hipEvent_t ev[8] = {};
    std::vector<hipEvent_t> band_ev;       // start/stop pairs of the passes of a query
};
void ctx_release(QueryCtx *q); // device memory and events (not the stream)
// Query scratch for a triangle buffer of cap records and kout results (query.hip).
int ensure_scratch(const tt_graph *g, QueryCtx *q, uint64_t cap, uint64_t kout);
// Marks (g->emark) the edges of `budget` weighted edge draws with exponent qexp (query.hip).
int es_mark_edges(tt_graph *g, QueryCtx *q, double qexp, uint64_t budget, uint64_t seed);
// The first N records of q->buf0 sorted by key (desc) and IDs; the best min(N, k) first in *res.
int select_records(QueryCtx *q, uint64_t N, uint32_t k, trec **res);
// Best min(N, k) of the first N records of q->buf0, scored for `mode`, copied to HOST out.
int finish_topk(QueryCtx *q, uint64_t N, uint32_t k, int mode, tt_triangle *out, uint32_t *n_out);
int ensure_in_csr(tt_graph *g, hipStream_t s);
int ensure_opos(tt_graph *g, hipStream_t s);
int ensure_weight_stream(tt_graph *g, hipStream_t s, uint32_t bin);
int ensure_sym(tt_graph *g, hipStream_t s);

// Entries in descending order of their bound m_p(w_uv, maxw(u), maxw(v)) (grouped by
// weight_bin of an integer >= it), for one p: the entries that can be the base of a triangle
// scoring >= t are the prefix of bins >= weight_bin(t).  Built on first use of p.
struct BoundOrder {
    bool valid = false;
    bool building = false; // reserved by the query building it
    uint64_t pb = 0, last_use = 0;
    int users = 0; // queries streaming (or building) it; never replaced while > 0
    uint32_t *src = nullptr, *col = nullptr, *wgt = nullptr, *pos = nullptr;
    std::vector<uint64_t> hist; // host: entries per bin
    std::vector<uint64_t> base; // host: first entry of each bin (bins descending)
};

// ----------------------------------------------------------------------------- graph
struct tt_graph {
    uint32_t n = 0;
    uint64_t m = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    int device = 0;
    // Degree-oriented CSR: an entry u->v exists iff (deg u, u) < (deg v, v).  Rows are laid out
    // in descending order of the row bound hb (grouped by weight_bin(hb)), so that the rows
    // that can hold a triangle of score >= t form a prefix of the entry arrays.
    uint64_t *rstart = nullptr; // [n+1] first entry of u's row
    uint32_t *rlen = nullptr;   // [n+1] out-degree of u
    uint32_t *col = nullptr;    // [m] head vertex v (original ID); rows sorted by v
    uint32_t *wgt = nullptr;    // [m] edge weight
    uint32_t *osrc = nullptr;   // [m] tail vertex u of each entry
    uint32_t *eid = nullptr;    // [m] input edge index of each entry
    uint32_t *opos = nullptr;   // [m] entry position of each input edge (built by the first sampling query)
    uint32_t *wcol = nullptr;   // [m] the same rows sorted by weight descending (then head ID)
    uint32_t *wwgt = nullptr;   // [m]
    uint32_t *wpos = nullptr;   // [m] position of each weight-sorted entry in the head-sorted row
    // The same entries in descending weight_bin(weight) order: for a band in which every edge
    // of a qualifying triangle must weigh >= z, the entries that can be its base are a prefix.
    uint32_t *ws_src = nullptr, *ws_col = nullptr, *ws_wgt = nullptr;
    uint32_t *ws_pos = nullptr; // head-sorted position of each such entry
    uint32_t *ws_hmx = nullptr; // row maximum of each such entry's head
    unsigned long long *ws_base = nullptr; // [WBINS] device copy of wbase
    std::atomic<uint32_t> ws_low{2048u}; // bins >= ws_low are in place (set after they are); 2048 = WBINS
    std::vector<uint64_t> wbase; // host: first entry of each weight bin (bins descending)
    uint32_t *maxw = nullptr;   // [n] largest weight in u's out-row (0 for an empty row)
    VInfo *vinfo = nullptr;     // [n+1] rstart, rlen, maxw packed (the intersection's reads)
    uint2 *cw = nullptr;        // [m] (col, wgt) interleaved: a binary-search hit holds the weight
    uint32_t *hmx = nullptr;    // [m] maxw of each entry's head: the filter's bound test streams it
                                //     instead of gathering maxw[v] at random
    uint32_t *hb = nullptr;     // [n] max(maxw[u], maxw[v] over out-neighbours v): bounds every
                                //     triangle based at u, for every p
    uint32_t *deg = nullptr;    // [n] undirected degree
    uint32_t *in_w = nullptr;   // [m] weights in input order (sampling prefix sums)
    // symmetric adjacency (rows sorted by neighbour), built by the first wedge or path sampling
    // query, with the per-row prefix sums of w^q of its most recent exponent
    uint64_t *srstart = nullptr; // [n+1]
    uint32_t *scol = nullptr;    // [2m]
    uint32_t *sw = nullptr;      // [2m]
    double *srowp = nullptr;     // [2m] inclusive prefix of w^q within each row
    double srow_q = -1.0;        // its exponent (-1: none)
    // transpose of the oriented CSR, built on the first subset query: for every head v, the
    // tails u of its in-entries u->v
    uint64_t *irstart = nullptr; // [n+2]
    uint32_t *itail = nullptr;
    std::mutex init_mu;
    uint32_t wmax = 0;          // largest weight in the graph
    uint32_t max_outdeg = 0;
    std::vector<uint64_t> whist; // host: edge count per weight_bin(w)
    std::vector<uint64_t> ebin;  // host: entry count per weight_bin(hb[tail])
    std::vector<uint64_t> ebase; // host: first entry of each bin (bins in descending order)
    uint64_t bytes = 0;
    QueryCtx q;                 // device state of the synchronous query calls
    uint8_t *emark = nullptr;   // [m] per-entry marks (sampling)
    // sampling tables, cached for the two most recent exponents q
    struct SampleTable {
        double q = -1.0;
        void *prefix = nullptr;   // u64 (q=1), u128 (q=2,3) or double (other q), [m]
        uint32_t *guide = nullptr; // [2^bits + 1] first candidate edge per top-bits bucket
        void *scan_tmp = nullptr;  // block sums of the prefix scan (scan_tmp_bytes(m))
        uint64_t last_use = 0;
    } tables[2];
    uint32_t guide_bits = 0;
    uint64_t use_clock = 0;
    std::mutex mu;
    BoundOrder bord[8];       // for the most recent p (guarded by init_mu)
    uint32_t max_orders = 8;
    uint64_t order_clock = 0;
    // entries streamed so far by queries of each recent p without a bound order: an order is
    // built once they exceed ORDER_AFTER times m (its cost is a few passes over the entries)
    struct StreamedAt {
        uint64_t pb = 0, entries = 0, last_use = 0;
    } streamed[16];
};

// ----------------------------------------------------------------------------- weight bins
// 2048 log-spaced bins: w < 64 exact; otherwise 64 bins per octave.
constexpr int WBINS = 2048;
static_assert(WBINS == 2048, "tt_graph::ws_low starts at WBINS");
__host__ __device__ inline uint32_t weight_bin(uint32_t w) {
    if (w < 64) return w;
    uint32_t e = 31u - (uint32_t)__builtin_clz(w);          // 6..31
    uint32_t top = w >> (e - 6);                            // 64..127
    return (e - 6) * 64u + top;                             // 64..1727
}
__host__ __device__ inline uint32_t weight_bin_low(uint32_t b) {
    if (b < 64) return b;
    uint32_t e = (b - 64) / 64 + 6, top = (b - 64) % 64 + 64;
    return top << (e - 6);
}

// ----------------------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess)                                                              \
            return fail(_e == hipErrorOutOfMemory ? TT_E_NOMEM : TT_E_DEVICE,              \
                        std::string(#expr) + ": " + hipGetErrorString(_e));                \
    } while (0)

int dev_alloc(tt_graph *g, void **p, size_t bytes);
size_t dev_round(size_t bytes);   // the size dev_alloc hands out for a request of `bytes`
size_t dev_bytes(const void *p);  // size of a live block from dev_alloc (0 if none)
void dev_free(tt_graph *g, void *p, size_t bytes);
int num_cus();

// ----------------------------------------------------------------------------- wave helpers
__device__ inline uint64_t wave_ballot(bool b) { return __ballot(b); }

template <typename T> __device__ inline T wave_incl_scan(T x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}
template <typename T> __device__ inline T wave_max(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T y = __shfl_xor(x, o, 64);
        x = x > y ? x : y;
    }
    return x;
}
template <typename T> __device__ inline T wave_sum(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// scan helpers (scan.hip)
// Exclusive prefix sums on stream s.  With tmp (at least scan_tmp_bytes(n) bytes, kept by the
// caller until the stream has run the scan) nothing is allocated and the call does not wait;
// without it the call waits for the scan.
uint64_t scan_tmp_bytes(uint64_t n);
int exclusive_scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, hipStream_t s, tt_graph *g,
                              void *tmp = nullptr);
