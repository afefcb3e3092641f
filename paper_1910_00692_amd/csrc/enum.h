// enum.h — the enumeration core shared by single-graph and batched queries: order keys of
// Eq. 1, the pruning bounds, and the filter / intersect kernels of one pass over a band of
// scores.
#pragma once
#include "common.h"

namespace {

// ----------------------------------------------------------------------------- scoring
__host__ __device__ __forceinline__ double u128_to_double(u128 x) {
    return (double)(uint64_t)(x >> 64) * 18446744073709551616.0 + (double)(uint64_t)x;
}

// The scoring and bound functions below are compiled for the host as well, so that their
// pruning properties can be checked on the CPU.
//
// Eq. 1 for a generic p, rewritten so that no power overflows and small |p| loses nothing:
// m = s * exp(log1p(mean(expm1(p * log(x/s)))) / p), s = max (p > 0) or min (p < 0).
__host__ __device__ inline double gen_mean(double p, double a, double b, double c) {
    const double s = p > 0.0 ? fmax(a, fmax(b, c)) : fmin(a, fmin(b, c));
    const double acc = expm1(p * log(a / s)) + expm1(p * log(b / s)) + expm1(p * log(c / s));
    return s * exp(log1p(acc / 3.0) / p);
}

__host__ __device__ __forceinline__ uint32_t max3(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t x = a > b ? a : b;
    return x > c ? x : c;
}
__host__ __device__ __forceinline__ uint32_t min3(uint32_t a, uint32_t b, uint32_t c) {
    const uint32_t x = a < b ? a : b;
    return x < c ? x : c;
}

// Order key of the integer modes (every mode but the generic p).
__host__ __device__ __forceinline__ u128 int_key(int mode, uint32_t a, uint32_t b, uint32_t c) {
    switch (mode) {
    case MODE_MAX: return (u128)max3(a, b, c);
    case MODE_MIN: return (u128)min3(a, b, c);
    case MODE_SUM: return (u128)((uint64_t)a + b + c);
    case MODE_SUMSQ: return (u128)((uint64_t)a * a) + (u128)((uint64_t)b * b) + (u128)((uint64_t)c * c);
    default: // MODE_PROD
        return (u128)((uint64_t)a * b) * (uint64_t)c;
    }
}

// The kernels of a pass are compiled twice: GEN for the generic p (FP64 bits of Eq. 1) and
// !GEN for the integer modes, which then carry none of the transcendental code (and need far
// fewer registers).
template <bool GEN>
__host__ __device__ __forceinline__ u128 score_key_t(int mode, double p, uint32_t a, uint32_t b, uint32_t c) {
    if (GEN) return (u128)__builtin_bit_cast(uint64_t, gen_mean(p, (double)a, (double)b, (double)c));
    return int_key(mode, a, b, c);
}

__host__ __device__ __forceinline__ u128 score_key(int mode, double p, uint32_t a, uint32_t b, uint32_t c) {
    return mode == MODE_GEN ? score_key_t<true>(mode, p, a, b, c) : int_key(mode, a, b, c);
}

__host__ __device__ inline double key_to_score(int mode, u128 key) {
    switch (mode) {
    case MODE_MAX:
    case MODE_MIN: return (double)(uint64_t)key;
    case MODE_SUM: return (double)(uint64_t)key / 3.0;
    case MODE_SUMSQ: return sqrt(u128_to_double(key) / 3.0);
    case MODE_PROD: return cbrt(u128_to_double(key));
    default: return __builtin_bit_cast(double, (uint64_t)key);
    }
}

__device__ __forceinline__ bool better(const trec &a, const trec &b) {
    if (a.khi != b.khi) return a.khi > b.khi;
    if (a.klo != b.klo) return a.klo > b.klo;
    if (a.i != b.i) return a.i < b.i;
    if (a.j != b.j) return a.j < b.j;
    return a.l < b.l;
}

// The record every real triangle beats (keys are >= 1).
__device__ __forceinline__ trec worst_rec() {
    trec r;
    r.khi = 0; r.klo = 0; r.i = r.j = r.l = 0xFFFFFFFFu; r.pad = 0;
    return r;
}

// ----------------------------------------------------------------------------- bounds
struct Band {
    u128 L;              // inclusive lower bound on the order key ...
    uint32_t Li, Lj, Ll; // ... and, at key == L, on (i, j, l) (all 0xFFFFFFFF: no restriction)
    u128 U;              // exclusive upper bound on the order key if hasU
    int hasU;
    int mode;
    double p;
    double theta;        // generic p: the score L as a double
};

// key(a, Wu, Wv) >= L : no triangle on this entry can reach the band otherwise
template <bool GEN>
__host__ __device__ __forceinline__ bool bound_ok(const Band &B, uint32_t a, uint32_t Wu, uint32_t Wv) {
    if (B.L == 0) return true;
    if (GEN) {
        // cheap upper bounds first: m_p <= max for every p, m_p <= arithmetic mean for p <= 1
        const double lim = B.theta * (1.0 - 1e-12);
        const double da = (double)a, du = (double)Wu, dv = (double)Wv;
        if (fmax(da, fmax(du, dv)) < lim) return false;
        if (B.p <= 1.0 && (da + du + dv) / 3.0 < lim * (1.0 - 1e-12)) return false;
        return gen_mean(B.p, da, du, dv) >= lim;
    }
    return int_key(B.mode, a, Wu, Wv) >= B.L;
}

// Smallest weight x (never above the exact one) with m_p(a, x, W) >= theta, generic p.
__host__ __device__ uint64_t gen_min_other(double p, double theta, double a, double W) {
    if (p > 0.0) {
        const double s = fmax(theta, fmax(a, W));
        const double t3 = 3.0 * pow(theta / s, p);
        double D = t3 - pow(a / s, p) - pow(W / s, p);
        D -= 1e-12 * (t3 + 2.0);
        if (!(D > 0.0)) return 0;
        const double x = s * pow(D, 1.0 / p) * (1.0 - 1e-9);
        return x < 1.0 ? 0 : (x >= 1.8e19 ? ~0ull : (uint64_t)floor(x));
    } else {
        const double s = fmin(theta, fmin(a, W));
        const double t3 = 3.0 * pow(theta / s, p);
        double D = t3 - pow(a / s, p) - pow(W / s, p);
        D += 1e-12 * (t3 + 2.0);
        if (!(D > 0.0)) return ~0ull;
        const double x = s * pow(D, 1.0 / p) * (1.0 - 1e-9);
        return x < 1.0 ? 0 : (x >= 1.8e19 ? ~0ull : (uint64_t)floor(x));
    }
}

// Smallest weight x (a lower bound of it) for which key(a, x, W) can still reach L.
template <bool GEN> __host__ __device__ __forceinline__ uint64_t min_other(const Band &B, uint32_t a, uint32_t W) {
    if (B.L == 0) return 0;
    if (GEN) return gen_min_other(B.p, B.theta, (double)a, (double)W);
    switch (B.mode) {
    case MODE_MAX: return ((u128)a >= B.L || (u128)W >= B.L) ? 0 : (uint64_t)B.L;
    case MODE_MIN: return (uint64_t)B.L;
    case MODE_SUM: {
        const uint64_t aw = (uint64_t)a + W, L = (uint64_t)B.L;
        return L > aw ? L - aw : 0;
    }
    case MODE_SUMSQ: {
        const u128 aw = (u128)((uint64_t)a * a) + (u128)((uint64_t)W * W);
        if (B.L <= aw) return 0;
        const uint64_t z = (uint64_t)sqrt(u128_to_double(B.L - aw));
        return z > 1 ? z - 1 : 0;
    }
    default: { // MODE_PROD
        const double q = u128_to_double(B.L) / ((double)a * (double)W);
        if (q <= 1.0) return 0;
        if (q >= 1.8e19) return ~0ull;
        const uint64_t z = (uint64_t)q;
        return z > 1 ? z - 1 : 0;
    }
    }
}

__device__ __forceinline__ bool in_band(const Band &B, u128 key, uint32_t i, uint32_t j, uint32_t l) {
    if (B.hasU && key >= B.U) return false;
    if (key != B.L) return key > B.L;
    return i < B.Li || (i == B.Li && (j < B.Lj || (j == B.Lj && l <= B.Ll)));
}

// ----------------------------------------------------------------------------- enumeration
enum { FILTER_NONE = 0, FILTER_EDGES = 1, FILTER_VERTICES = 2 };
// FL_PAIRS: a FL_REQ_C candidate whose iterated side is the run of u's heads in the subset
// (EnumArgs::sp_*), not a prefix of u's weight-sorted row; qB then holds that side's floor.
enum { FL_MARK_UV = 1, FL_REQ_A = 2, FL_REQ_B = 4, FL_REQ_C = 8, FL_PAIRS = 16 };
// Admissible entries of the other row scanned instead of a binary search (EnumArgs::scan_max).
constexpr uint32_t SCAN_MAX = 32;

struct EnumArgs {
    const uint64_t *rstart;
    const uint32_t *rlen, *col, *wgt, *wcol, *wwgt, *wpos, *maxw;
    const VInfo *vi; // rstart, rlen, maxw per vertex
    const uint2 *cw; // (col, wgt) per entry
    // a candidate whose two rows hold at most this many entries together is intersected by one
    // lane merging the two head-sorted rows; longer ones by the wave's binary searches
    uint32_t merge_max;
    // an entry of the iterated row is looked up in the other row by scanning that row's
    // admissible entries (the leading ones of its weight-sorted copy) when there are at most
    // this many and the scan takes no more steps than a binary search of the head-sorted row
    uint32_t scan_max;
    // the stream of candidate entries (tail, head, weight, head-sorted position or NULL if the
    // stream is the head-sorted layout itself) and its length
    const uint32_t *s_src, *s_col, *s_wgt, *s_pos;
    const uint32_t *s_hmx; // maxw of each stream entry's head (single-graph streams), else NULL
    uint64_t E;
    uint64_t pos_off; // head-sorted position of stream entry 0 when s_pos is NULL
    const unsigned long long *skip; // set (between passes) once the answer is complete
    Band B;
    const uint8_t *emark;  // FILTER_EDGES: drawn entries (head-sorted positions)
    const uint8_t *vflag;  // FILTER_EDGES: vertex has a drawn out-entry; FILTER_VERTICES: vertex in subset
    const uint8_t *vflag2; // FILTER_VERTICES: vertex has an out-neighbour in the subset
    // FILTER_VERTICES on the compact stream: for the listed in-neighbour with index i (the
    // stream's position field), its heads in the subset and their weights are
    // sp_c / sp_w[sp_start[i] .. sp_start[i] + sp_cnt[i]); NULL elsewhere
    const uint32_t *sp_c, *sp_w, *sp_start, *sp_cnt;
    trec *out;
    unsigned long long *count;
    uint64_t cap;
    // per-pass counters, each spread over STAT_SLOTS slots to avoid same-address atomics:
    // [0] candidates [1] intersected entries [2] emitted [3] streamed [4] passes
    unsigned long long *stats;
    // candidate list: block b of the filter writes its candidates to C[b*seg ...] and their
    // number to ccnt[b]
    cand *C;
    uint32_t *ccnt;
    uint64_t seg;
    uint32_t nseg;
    // candidates with more than heavy_min entries to intersect go to heavy[] and their
    // HEAVY_PIECE-entry pieces to hpiece[] (counts in nheavy[0], nheavy[1], cleared by the
    // filter) for k_intersect_heavy; heavy == NULL keeps them in-wave
    Heavy *heavy;
    unsigned long long *nheavy;
    uint2 *hpiece;
    uint32_t heavy_min;
    unsigned long long *hstat; // [0] heavy candidates spread, [1] beyond the list (or NULL)
    // batched form (one disjoint union of graphs): the stream is the concatenation, over the
    // graphs, of the first E_g entries of graph g's weight-ordered segment, which starts at
    // goff[g]; poff is the exclusive prefix of E_g (ng + 1 values, poff[ng] = the length,
    // read on the device).  Graph g's band is bands[g]; its triangles go to out[g*R ...] with
    // their number in gcount[g].  Candidates carry their graph in `pos`.
    const Band *bands;
    const uint64_t *poff, *goff;
    uint32_t ng;
    unsigned long long *gcount;
    uint32_t R;
};

constexpr int STAT_SLOTS = 1024;
__device__ __forceinline__ void stat_add(unsigned long long *stats, int c, unsigned long long v) {
    if (v) atomicAdd(&stats[c * STAT_SLOTS + (blockIdx.x & (STAT_SLOTS - 1))], v);
}

// Number of entries of a weight-sorted (descending) row with weight >= z.
__device__ __forceinline__ uint32_t count_at_least(const uint32_t *ww, uint64_t b, uint32_t len, uint64_t z) {
    if (z == 0) return len;
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)ww[b + mid] >= z) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Number of entries of two weight-sorted rows at or above their floors; both binary searches
// advance together so that their loads overlap.
// q1, q2 = the number of entries of each weight-descending row with weight >= its floor (a
// floor of 0 counts the whole row).  Those entries lead their rows, and there are usually few,
// so each count is found by galloping from the row's start (probes at 0, 2, 6, 14, ...) and
// then a binary search between the last two probes: a handful of loads from the row's first
// lines instead of a search over the whole row.  The two searches are interleaved.
__device__ __forceinline__ void count_pair(const uint32_t *ww, uint64_t b1, uint32_t n1, uint64_t z1, uint64_t b2,
                                           uint32_t n2, uint64_t z2, uint32_t &q1, uint32_t &q2) {
    // the count lies in [lo, up]: entries before lo reach the floor, entries from up on do not
    uint32_t lo1 = z1 ? 0 : n1, up1 = n1, lo2 = z2 ? 0 : n2, up2 = n2, s1 = 1, s2 = 1;
    bool g1 = lo1 < up1, g2 = lo2 < up2;
    while (g1 || g2) {
        if (g1) {
            const uint32_t i = lo1 + s1 - 1;
            if (i >= up1) g1 = false;
            else if ((uint64_t)ww[b1 + i] >= z1) { lo1 = i + 1; s1 <<= 1; }
            else { up1 = i; g1 = false; }
        }
        if (g2) {
            const uint32_t i = lo2 + s2 - 1;
            if (i >= up2) g2 = false;
            else if ((uint64_t)ww[b2 + i] >= z2) { lo2 = i + 1; s2 <<= 1; }
            else { up2 = i; g2 = false; }
        }
    }
    while (lo1 < up1 || lo2 < up2) {
        if (lo1 < up1) {
            const uint32_t mid = (lo1 + up1) >> 1;
            if ((uint64_t)ww[b1 + mid] >= z1) lo1 = mid + 1; else up1 = mid;
        }
        if (lo2 < up2) {
            const uint32_t mid = (lo2 + up2) >> 1;
            if ((uint64_t)ww[b2 + mid] >= z2) lo2 = mid + 1; else up2 = mid;
        }
    }
    q1 = lo1;
    q2 = lo2;
}

constexpr int FILTER_UNROLL = 4;

// Phase 1: stream the first E entries of the chosen order; an entry that can be the base of a
// triangle in the band (bound test + subset / sampling pre-test) is appended to the candidate
// list (wave ballot, one atomic per wave).  Pure streaming: FILTER_UNROLL entries per lane
// are in flight at once.
// The length of the stream and of a block's segment (batched form: read on the device).
template <bool BATCH> __device__ __forceinline__ void stream_extent(const EnumArgs &A, uint64_t &E, uint64_t &seg) {
    if (BATCH) {
        E = A.poff[A.ng];
        seg = (E + A.nseg - 1) / A.nseg;
    } else {
        E = A.E;
        seg = A.seg;
    }
}

// Batched form: the last graph in [lo, hi) with poff[g] <= e, given poff[lo] <= e < poff[hi]
// (graphs streaming nothing share their offset with the next one, so it is the graph whose
// part of the stream holds e).
__device__ __forceinline__ uint32_t graph_bsearch(const uint64_t *poff, uint32_t lo, uint32_t hi, uint64_t e) {
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (poff[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// Batched form: the graph of stream index e (< poff[ng]), moving forward from a graph g at or
// before it by galloping, so that runs of graphs streaming few entries cost a logarithm.
__device__ __forceinline__ uint32_t graph_at(const uint64_t *poff, uint32_t ng, uint32_t g, uint64_t e) {
    if (poff[g + 1] > e) return g;
    uint32_t lo = g + 1, step = 1, hi;
    for (;;) {
        hi = lo + step;
        if (hi >= ng) { hi = ng; break; }
        if (poff[hi] > e) break;
        lo = hi;
        step <<= 1;
    }
    return graph_bsearch(poff, lo, hi, e);
}

// Batched form: the graph whose part of the stream holds e.
__device__ __forceinline__ uint32_t graph_search(const uint64_t *poff, uint32_t ng, uint64_t e) {
    return graph_bsearch(poff, 0, ng, e);
}

template <int FILTER, bool BATCH, bool GEN> __global__ __launch_bounds__(256) void k_filter(EnumArgs A) {
    __shared__ uint32_t lcount;
    // the previous piece's intersect kernels have finished (stream order)
    if (A.nheavy && blockIdx.x == 0 && threadIdx.x == 0) A.nheavy[0] = A.nheavy[1] = 0;
    if (A.skip && *A.skip) return; // written only between passes
    uint64_t E, seg;
    stream_extent<BATCH>(A, E, seg);
    if (threadIdx.x == 0) lcount = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        stat_add(A.stats, 3, E);
        stat_add(A.stats, 4, 1);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint64_t lo = (uint64_t)blockIdx.x * seg;
    const uint64_t hi = lo + seg < E ? lo + seg : E;
    cand *out = A.C + lo;
    uint32_t gcur = 0; // batched form: graph of this lane's latest entry
    if (BATCH && lo < hi) gcur = graph_search(A.poff, A.ng, lo);
    for (uint64_t base = lo + (threadIdx.x >> 6) * 64 * FILTER_UNROLL; base < hi; base += blockDim.x * FILTER_UNROLL) {
        uint32_t u[FILTER_UNROLL], v[FILTER_UNROLL], a[FILTER_UNROLL], pos[FILTER_UNROLL], mv[FILTER_UNROLL];
        bool pass[FILTER_UNROLL];
#pragma unroll
        for (int k = 0; k < FILTER_UNROLL; k++) {
            const uint64_t e = base + (uint64_t)k * 64 + lane;
            pass[k] = e < hi;
            u[k] = v[k] = a[k] = pos[k] = mv[k] = 0;
            if (pass[k]) {
                uint64_t x = e;
                if (BATCH) {
                    gcur = graph_at(A.poff, A.ng, gcur, e);
                    x = A.goff[gcur] + (e - A.poff[gcur]);
                    pos[k] = gcur;
                }
                u[k] = A.s_src[x];
                v[k] = A.s_col[x];
                a[k] = A.s_wgt[x];
                if (!BATCH && A.s_hmx) mv[k] = A.s_hmx[x];
                // the entry position is needed only by the drawn-entry marks; the subset's
                // compact stream holds the tail's index in the list of in-neighbours there
                if (!BATCH && FILTER == FILTER_EDGES) pos[k] = A.s_pos ? A.s_pos[e] : (uint32_t)(e + A.pos_off);
                if (!BATCH && FILTER == FILTER_VERTICES && A.sp_c) pos[k] = A.s_pos[e];
            }
        }
        uint32_t n_pass = 0, rank[FILTER_UNROLL];
#pragma unroll
        for (int k = 0; k < FILTER_UNROLL; k++) {
            if (pass[k]) {
                bool pre = true;
                if (FILTER == FILTER_EDGES) pre = A.emark[pos[k]] || A.vflag[u[k]] || A.vflag[v[k]];
                else if (FILTER == FILTER_VERTICES)
                    pre = A.vflag[u[k]] || A.vflag[v[k]] || (A.vflag2[u[k]] && A.vflag2[v[k]]);
                if (BATCH) pass[k] = bound_ok<GEN>(A.bands[pos[k]], a[k], A.maxw[u[k]], A.maxw[v[k]]);
                else pass[k] = pre && bound_ok<GEN>(A.B, a[k], A.maxw[u[k]], A.s_hmx ? mv[k] : A.maxw[v[k]]);
            }
            const uint64_t bal = __ballot(pass[k]);
            rank[k] = n_pass + __popcll(bal & ((1ull << lane) - 1ull));
            n_pass += __popcll(bal);
        }
        if (n_pass) {
            uint32_t b0 = 0;
            if (lane == 0) b0 = atomicAdd(&lcount, n_pass); // LDS atomic: block-local offset
            b0 = __shfl(b0, 0, 64);
#pragma unroll
            for (int k = 0; k < FILTER_UNROLL; k++)
                if (pass[k]) out[b0 + rank[k]] = cand{u[k], v[k], a[k], pos[k]};
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        A.ccnt[blockIdx.x] = lcount;
        stat_add(A.stats, 0, lcount);
    }
}

// Phase 2: persistent waves over the candidate list (its length is read on the device).  A
// candidate u->v gets the weight floors zu (for w_uc) and zv (for w_vc); the entries of each
// row at or above its floor are a prefix of the weight-sorted copy of the row.  The side with
// fewer such entries is iterated: the wave flattens the (candidate, qualifying element) pairs
// of its 64 candidates across its lanes, and each lane binary-searches its element in the
// other row's head-sorted copy.
constexpr int MAX_SEG = 4096;

// The triangle (u, v, c) with weights a = w_uv, x = w_uc, y = w_vc as a record, and whether it
// lies in its band.
template <bool BATCH, bool GEN>
__device__ __forceinline__ bool make_rec(const EnumArgs &A, uint32_t g, uint32_t a, uint32_t x, uint32_t y,
                                         uint32_t u, uint32_t v, uint32_t c, trec &r);

// Appends the records of the lanes with ok set: one ballot and one global atomic per wave (per
// graph present among the lanes in the batched form).
template <bool BATCH>
__device__ __forceinline__ void wave_emit(const EnumArgs &A, bool ok, const trec &r, uint32_t og, int lane,
                                          unsigned long long &s_emit) {
    const uint64_t bal = __ballot(ok);
    if (BATCH && bal) {
        if (lane == 0) s_emit += __popcll(bal);
        uint64_t pend = bal;
        while (pend) {
            const int lead = __ffsll((unsigned long long)pend) - 1;
            const uint32_t gl = __shfl(og, lead, 64);
            const bool mine = ok && og == gl;
            const uint64_t grp = __ballot(mine);
            unsigned long long b0 = 0;
            if (lane == lead) b0 = atomicAdd(&A.gcount[gl], (unsigned long long)__popcll(grp));
            b0 = __shfl(b0, lead, 64);
            const uint64_t slot = b0 + __popcll(grp & ((1ull << lane) - 1ull));
            if (mine && slot < A.R) A.out[(uint64_t)gl * A.R + slot] = r;
            pend &= ~grp;
        }
    } else if (bal) {
        const uint32_t nb = __popcll(bal);
        unsigned long long b0 = 0;
        if (lane == 0) b0 = atomicAdd(A.count, (unsigned long long)nb);
        b0 = __shfl(b0, 0, 64);
        const uint32_t rank = __popcll(bal & ((1ull << lane) - 1ull));
        if (ok && b0 + rank < A.cap) A.out[b0 + rank] = r;
        if (lane == 0) s_emit += nb;
    }
}

template <bool BATCH> __device__ __forceinline__ const Band &band_of(const EnumArgs &A, uint32_t g) {
    if (BATCH) return A.bands[g];
    return A.B;
}

template <bool BATCH, bool GEN>
__device__ __forceinline__ bool make_rec(const EnumArgs &A, uint32_t g, uint32_t a, uint32_t x, uint32_t y,
                                         uint32_t u, uint32_t v, uint32_t c, trec &r) {
    const u128 key = score_key_t<GEN>(A.B.mode, A.B.p, a, x, y);
    uint32_t i = u, j = v, l = c, tmp;
    if (i > j) { tmp = i; i = j; j = tmp; }
    if (j > l) { tmp = j; j = l; l = tmp; }
    if (i > j) { tmp = i; i = j; j = tmp; }
    r.khi = (uint64_t)(key >> 64);
    r.klo = (uint64_t)key;
    r.i = i; r.j = j; r.l = l; r.pad = 0;
    return in_band(band_of<BATCH>(A, g), key, i, j, l);
}

// Entry pa of a candidate's iterated row (weight-sorted copy: head c, weight x) looked up in the
// other row: scanned among that row's qB admissible entries (the leading ones of its
// weight-sorted copy) when there are at most scan_max and the scan is no longer than the
// search, else binary-searched in its head-sorted copy (Blen entries from Bb) and then held to
// the floor zB.  True with the triangle's record
// when it is admissible and lies in its band.
template <int FILTER, bool BATCH, bool GEN>
__device__ __forceinline__ bool lookup_entry(const EnumArgs &A, uint64_t pa, uint64_t Bb, uint32_t Blen, uint32_t qB,
                                             uint32_t zB, uint32_t a, uint32_t u, uint32_t v, uint32_t fl,
                                             uint32_t g, trec &r) {
    if (FILTER == FILTER_VERTICES && (fl & FL_PAIRS)) {
        // a head c of u in the subset (weight x >= the floor kept in qB), looked up in v's
        // head-sorted row
        const uint32_t c = A.sp_c[pa], x = A.sp_w[pa];
        if (x < qB) return false;
        uint64_t lo = Bb, hi = Bb + Blen;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (A.cw[mid].x < c) lo = mid + 1; else hi = mid;
        }
        const uint2 hit = lo < Bb + Blen ? A.cw[lo] : make_uint2(~0u, 0u);
        if (hit.x != c || hit.y < zB) return false;
        return make_rec<BATCH, GEN>(A, g, a, x, hit.y, u, v, c, r);
    }
    const uint32_t c = A.wcol[pa], x = A.wwgt[pa];
    if (FILTER == FILTER_VERTICES && (fl & FL_REQ_C) && !A.vflag[c]) return false;
    uint8_t markA = 0;
    if (FILTER == FILTER_EDGES) {
        markA = A.emark[A.wpos[pa]];
        if ((fl & FL_REQ_A) && !markA) return false;
    }
    // the scan issues four independent loads per step; it is taken when it needs no more
    // steps than the binary search has levels
    if (qB <= A.scan_max && (qB + 3) / 4 <= 32u - (uint32_t)__clz(Blen)) {
        uint32_t hit = qB;
        for (uint32_t t = 0; t < qB; t += 4) {
            const uint32_t c0 = A.wcol[Bb + t], c1 = t + 1 < qB ? A.wcol[Bb + t + 1] : ~0u,
                           c2 = t + 2 < qB ? A.wcol[Bb + t + 2] : ~0u, c3 = t + 3 < qB ? A.wcol[Bb + t + 3] : ~0u;
            if (c0 == c) { hit = t; break; }
            if (c1 == c) { hit = t + 1; break; }
            if (c2 == c) { hit = t + 2; break; }
            if (c3 == c) { hit = t + 3; break; }
        }
        if (hit == qB) return false;
        if (FILTER == FILTER_EDGES) {
            const uint8_t markB = A.emark[A.wpos[Bb + hit]];
            if ((fl & FL_REQ_B) && !markB) return false;
            if (!((fl & FL_MARK_UV) || markA || markB)) return false;
        }
        return make_rec<BATCH, GEN>(A, g, a, x, A.wwgt[Bb + hit], u, v, c, r);
    }
    uint64_t lo = Bb, hi = Bb + Blen;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (A.cw[mid].x < c) lo = mid + 1; else hi = mid;
    }
    const uint2 hit = lo < Bb + Blen ? A.cw[lo] : make_uint2(~0u, 0u);
    if (hit.x != c || hit.y < zB) return false;
    if (FILTER == FILTER_EDGES) {
        const uint8_t markB = A.emark[lo];
        if ((fl & FL_REQ_B) && !markB) return false;
        if (!((fl & FL_MARK_UV) || markA || markB)) return false;
    }
    return make_rec<BATCH, GEN>(A, g, a, x, hit.y, u, v, c, r);
}

// Block-wide exclusive prefix of per-item counts: pre[i] = sum of cnt(j) for j < i, over
// N = 256 * PER items (each thread owns PER consecutive ones); pre[N] = the total.
template <int PER, typename F> __device__ __forceinline__ void block_prefix(uint32_t *pre, uint32_t *wsum, F cnt) {
    const int lane = threadIdx.x & 63;
    uint32_t loc[PER], sum = 0;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        loc[i] = cnt(threadIdx.x * PER + i);
        sum += loc[i];
    }
    const uint32_t incl = wave_incl_scan(sum);
    if (lane == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < (int)(threadIdx.x >> 6); w++) run += wsum[w];
#pragma unroll
    for (int i = 0; i < PER; i++) {
        pre[threadIdx.x * PER + i] = run;
        run += loc[i];
    }
    if (threadIdx.x == 255) pre[256 * PER] = run;
    __syncthreads();
}

// The last i with pre[i] <= x, over pre[0 .. n] (pre[0] = 0 <= x).
__device__ __forceinline__ uint32_t prefix_owner(const uint32_t *pre, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

template <int FILTER, bool BATCH, bool GEN> __global__ __launch_bounds__(256) void k_intersect(EnumArgs A) {
    __shared__ uint32_t pre[MAX_SEG + 1]; // exclusive prefix of 64-candidate chunks per segment
    __shared__ uint32_t wsum[4];
    if (A.skip && *A.skip) return;
    uint64_t E_unused, seg;
    stream_extent<BATCH>(A, E_unused, seg);
    const int lane = threadIdx.x & 63;
    block_prefix<(MAX_SEG + 255) / 256>(pre, wsum, [&](uint32_t sg) -> uint32_t {
        return sg < A.nseg ? (A.ccnt[sg] + 63) >> 6 : 0;
    });
    const uint32_t nchunks = pre[MAX_SEG];
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long s_inter = 0, s_emit = 0;
    for (uint64_t ch = wave; ch < nchunks; ch += nwaves) {
        const uint32_t sg = prefix_owner(pre, MAX_SEG, (uint32_t)ch);
        const uint64_t j = ((uint64_t)(ch - pre[sg]) << 6) + (uint64_t)lane;
        bool pass = false, merge = false;
        // per lane: its candidate, and either the search plan (iterated row Ab with qA
        // admissible entries, other row Bb) or the two rows to merge (Ab/ul with floor zA,
        // Bb/Blen with floor zB)
        uint32_t a = 0, u = 0, v = 0, qA = 0, qB = 0, Blen = 0, zA = 0, zB = 0, fl = 0, g = 0;
        uint64_t Ab = 0, Bb = 0;
        if (j < A.ccnt[sg]) {
            const cand c = A.C[(uint64_t)sg * seg + j];
            u = c.u;
            v = c.v;
            a = c.a;
            if (BATCH) g = c.pos;
            const Band &B = band_of<BATCH>(A, g);
            const VInfo iu = A.vi[u], iv = A.vi[v];
            const uint32_t Wu = iu.maxw, Wv = iv.maxw;
            const uint64_t ub = iu.rstart, vb = iv.rstart;
            const uint32_t ul = iu.rlen, vl = iv.rlen;
            if (FILTER == FILTER_EDGES && A.emark[c.pos]) fl |= FL_MARK_UV;
            if (FILTER == FILTER_VERTICES && !A.vflag[u] && !A.vflag[v]) fl |= FL_REQ_C;
            const uint64_t zu = min_other<GEN>(B, a, Wv), zv = min_other<GEN>(B, a, Wu);
            pass = zu <= Wu && zv <= Wv; // then both floors fit 32 bits
            // a triangle of a candidate with neither end in the subset must close on a subset
            // vertex: with the subset's lists, only u's heads in the subset are looked up
            const bool pairs = FILTER == FILTER_VERTICES && (fl & FL_REQ_C) && A.sp_c != nullptr;
            if (pass && pairs) {
                const uint32_t li = c.pos;
                Ab = A.sp_start[li];
                qA = A.sp_cnt[li];
                qB = (uint32_t)zu; // the floor of w_uc
                Bb = vb;
                Blen = vl;
                zB = (uint32_t)zv;
                fl |= FL_PAIRS;
                if (qA == 0) pass = false;
            }
            if (pass && !pairs && ul + vl <= A.merge_max) {
                merge = true;
                pass = false;
                Ab = ub; qA = ul; zA = (uint32_t)zu;
                Bb = vb; Blen = vl; zB = (uint32_t)zv;
            }
            if (pass && !pairs) {
                uint32_t qu, qv;
                count_pair(A.wwgt, ub, ul, zu, vb, vl, zv, qu, qv);
                const bool uA = qu <= qv;
                qA = uA ? qu : qv;
                qB = uA ? qv : qu;
                Ab = uA ? ub : vb;
                Bb = uA ? vb : ub;
                Blen = uA ? vl : ul;
                zB = (uint32_t)(uA ? zv : zu);
                if (qu == 0 || qv == 0) pass = false;
                if (FILTER == FILTER_EDGES && !(fl & FL_MARK_UV)) {
                    // a drawn edge must be one of the other two
                    const bool fa = A.vflag[uA ? u : v], fb = A.vflag[uA ? v : u];
                    if (!fa && !fb) pass = false;
                    if (!fb) fl |= FL_REQ_A; // only drawn entries of the iterated row can help
                    if (!fa) fl |= FL_REQ_B;
                }
            }
            if (pass && qA > A.heavy_min && A.heavy) {
                // reserve a record and the pieces; a range reserved past the list's end is
                // marked empty and the candidate stays with its wave
                const unsigned long long h = atomicAdd(A.nheavy, 1ull);
                bool spread = false;
                if (h < HEAVY_CAP) {
                    const uint32_t np = (qA + HEAVY_PIECE - 1) / HEAVY_PIECE;
                    const unsigned long long p0 = atomicAdd(A.nheavy + 1, (unsigned long long)np);
                    if (p0 + np <= HEAVY_PIECES) {
                        A.heavy[h] = Heavy{Ab, Bb, qA, qB, Blen, zB, a, u, v, fl, g, 0u};
                        for (uint32_t k2 = 0; k2 < np; k2++)
                            A.hpiece[p0 + k2] = make_uint2((uint32_t)h, k2);
                        spread = true;
                        pass = false; // its entries are intersected by k_intersect_heavy
                    } else {
                        for (unsigned long long k2 = p0; k2 < HEAVY_PIECES; k2++)
                            A.hpiece[k2] = make_uint2(~0u, 0u);
                    }
                }
                if (A.hstat) atomicAdd(A.hstat + (spread ? 0 : 1), 1ull);
            }
        }
        const uint32_t work = pass ? qA : 0;
        const uint32_t incl = wave_incl_scan(work);
        const uint32_t total = __shfl(incl, 63, 64);
        if (lane == 0) s_inter += total;
        for (uint32_t base = 0; base < total; base += 64) {
            const uint32_t t = base + (uint32_t)lane;
            const uint32_t tt = t < total ? t : total - 1;
            int s = 0; // owner lane: number of lanes whose inclusive end is <= tt
#pragma unroll
            for (int st = 32; st > 0; st >>= 1) {
                const uint32_t im = __shfl(incl, s + st - 1, 64);
                if (im <= tt) s += st;
            }
            const uint32_t o_incl = __shfl(incl, s, 64), o_work = __shfl(work, s, 64);
            const uint64_t oAb = __shfl(Ab, s, 64), oBb = __shfl(Bb, s, 64);
            const uint32_t oBlen = __shfl(Blen, s, 64), oqB = __shfl(qB, s, 64), ozB = __shfl(zB, s, 64),
                           oa = __shfl(a, s, 64), ou = __shfl(u, s, 64), ov = __shfl(v, s, 64),
                           ofl = __shfl(fl, s, 64);
            const uint32_t og = BATCH ? __shfl(g, s, 64) : 0u;
            bool ok = false;
            trec r;
            if (t < total)
                ok = lookup_entry<FILTER, BATCH, GEN>(A, oAb + (tt - (o_incl - o_work)), oBb, oBlen, oqB, ozB, oa, ou,
                                                      ov, ofl, og, r);
            wave_emit<BATCH>(A, ok, r, og, lane, s_emit);
        }
        // short rows: each such lane merges the two head-sorted rows (weights below their
        // floors skipped), one step per iteration, emitting with the whole wave
        const uint32_t msteps = wave_max(merge ? qA + Blen : 0u);
        uint32_t mi = 0, mj = 0;
        for (uint32_t step = 0; step < msteps; step++) {
            bool ok = false;
            trec r;
            if (merge && mi < qA && mj < Blen) {
                const uint2 xu = A.cw[Ab + mi], xv = A.cw[Bb + mj];
                if (xu.x < xv.x) {
                    mi++;
                } else if (xv.x < xu.x) {
                    mj++;
                } else {
                    const uint32_t c = xu.x;
                    bool adm = xu.y >= zA && xv.y >= zB;
                    if (FILTER == FILTER_VERTICES && (fl & FL_REQ_C)) adm = adm && A.vflag[c];
                    if (FILTER == FILTER_EDGES)
                        adm = adm && ((fl & FL_MARK_UV) || A.emark[Ab + mi] || A.emark[Bb + mj]);
                    if (adm) ok = make_rec<BATCH, GEN>(A, g, a, xu.y, xv.y, u, v, c, r);
                    mi++;
                    mj++;
                }
            }
            wave_emit<BATCH>(A, ok, r, g, lane, s_emit);
        }
        const uint32_t consumed = wave_sum(merge ? mi + mj : 0u);
        if (lane == 0) s_inter += consumed;
    }
    if (lane == 0) {
        stat_add(A.stats, 1, s_inter);
        stat_add(A.stats, 2, s_emit);
    }
}

// The heavy candidates of a piece: each was cut into HEAVY_PIECE-entry pieces of its iterated
// row when it was listed, and the waves of the grid take the pieces in turn, so that one long
// row is intersected by many waves at once instead of serialising the wave that found it.
template <int FILTER, bool BATCH, bool GEN> __global__ __launch_bounds__(256) void k_intersect_heavy(EnumArgs A) {
    if (A.skip && *A.skip) return;
    const unsigned long long np_all = A.nheavy[1];
    const uint32_t npieces = np_all < HEAVY_PIECES ? (uint32_t)np_all : HEAVY_PIECES;
    if (npieces == 0) return;
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long s_inter = 0, s_emit = 0;
    for (uint64_t pc = wave; pc < npieces; pc += nwaves) {
        const uint2 pe = A.hpiece[pc];
        if (pe.x == ~0u) continue; // reserved past the list's end, never filled
        const Heavy H = A.heavy[pe.x];
        const uint32_t t0 = pe.y * HEAVY_PIECE;
        const uint32_t t1 = min(t0 + HEAVY_PIECE, H.qA);
        if (lane == 0) s_inter += t1 - t0;
        for (uint32_t base = t0; base < t1; base += 64) {
            const uint32_t t = base + (uint32_t)lane;
            bool ok = false;
            trec r;
            if (t < t1)
                ok = lookup_entry<FILTER, BATCH, GEN>(A, H.Ab + t, H.Bb, H.Blen, H.qB, H.zB, H.a, H.u, H.v, H.fl,
                                                      H.g, r);
            wave_emit<BATCH>(A, ok, r, H.g, lane, s_emit);
        }
    }
    if (lane == 0) {
        stat_add(A.stats, 1, s_inter);
        stat_add(A.stats, 2, s_emit);
    }
}

// Sums the spread counters into out[0..5) and clears them.
__global__ void k_reduce_stats(unsigned long long *stats, unsigned long long *out) {
    const int c = blockIdx.x;
    unsigned long long v = 0;
    for (int t = threadIdx.x; t < STAT_SLOTS; t += blockDim.x) {
        v += stats[c * STAT_SLOTS + t];
        stats[c * STAT_SLOTS + t] = 0;
    }
    v = wave_sum(v);
    __shared__ unsigned long long ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[c] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Between two passes enqueued without a count read: the later bands are skipped once the
// buffer holds `need` triangles (the host then reads the count: the answer is complete, or the
// next threshold follows from it); *last records the last band allowed to run.
__global__ void k_band_gate(const unsigned long long *count, unsigned long long need, unsigned long long *skip,
                            unsigned long long band, unsigned long long *last) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || *skip) return;
    if (*count >= need) *skip = 1;
    else *last = band;
}

// An integer >= the score of every triangle based at entry u->v (m_p of the entry's weight
// and the two row maxima), at most the largest of the three.
__host__ __device__ __forceinline__ uint32_t entry_bound(int mode, double p, uint32_t a, uint32_t Wu, uint32_t Wv) {
    const uint32_t mx = max3(a, Wu, Wv);
    const double sc = key_to_score(mode, score_key(mode, p, a, Wu, Wv));
    const double up = ceil(sc * (1.0 + 1e-9));
    return up >= (double)mx ? mx : (uint32_t)up;
}

// ----------------------------------------------------------------------------- thresholds
// The order key of a triangle whose three weights all equal t.
__host__ __device__ inline u128 key_of_uniform(int mode, uint32_t t) {
    switch (mode) {
    case MODE_MAX:
    case MODE_MIN: return t;
    case MODE_SUM: return (u128)3 * t;
    case MODE_SUMSQ: return (u128)3 * ((uint64_t)t * t);
    case MODE_PROD: return (u128)((uint64_t)t * t) * t;
    default: {
        return (u128)__builtin_bit_cast(uint64_t, (double)t);
    }
    }
}

__host__ __device__ inline double key_as_double(u128 L) { return __builtin_bit_cast(double, (uint64_t)L); }

// The lightest edge of any triangle whose key is >= L weighs at least this (a lower bound):
// with the other two edges at the graph's largest weight W, key(W, W, z) must still reach L.
__host__ __device__ inline uint64_t weight_floor(int mode, double p, u128 L, uint32_t W) {
    if (L == 0) return 0;
    switch (mode) {
    case MODE_MAX: return 0;
    case MODE_MIN: return (uint64_t)L;
    case MODE_SUM: {
        const u128 w2 = (u128)2 * W;
        return L > w2 ? (uint64_t)(L - w2) : 0;
    }
    case MODE_SUMSQ: {
        const u128 w2 = (u128)2 * ((uint64_t)W * W);
        if (L <= w2) return 0;
        const uint64_t z = (uint64_t)sqrt(u128_to_double(L - w2));
        return z > 1 ? z - 1 : 0;
    }
    case MODE_PROD: {
        const double q = u128_to_double(L) / ((double)W * (double)W);
        if (q <= 1.0) return 0;
        const uint64_t z = q >= 1.8e19 ? ~0ull : (uint64_t)q;
        return z > 1 ? z - 1 : 0;
    }
    default: return gen_min_other(p, key_as_double(L), (double)W, (double)W);
    }
}

// An integer t <= the score of any triangle whose key is >= L (so rows with hb < t can be
// skipped): the score of key L, rounded down, lowered once more for the inexact roots.
__host__ __device__ inline uint64_t score_floor(int mode, u128 L) {
    if (L == 0) return 0;
    double v;
    switch (mode) {
    case MODE_MAX:
    case MODE_MIN: return (uint64_t)L;
    case MODE_SUM: return (uint64_t)(L / 3);
    case MODE_SUMSQ: v = sqrt(u128_to_double(L) / 3.0); break;
    case MODE_PROD: v = cbrt(u128_to_double(L)); break;
    default: v = key_as_double(L) * (1.0 - 1e-9); break;
    }
    if (!(v > 1.0)) return 0;
    const uint64_t f = (uint64_t)floor(v);
    return f > 0 ? f - 1 : 0;
}

} // namespace
