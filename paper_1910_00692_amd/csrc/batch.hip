// batch.hip — the batched form: one top-k per graph for many independent graphs of uneven
// size (the problem of Sec. 1 solved once per graph), in one captured launch sequence.
//
// Layout.  The graphs are loaded as one disjoint union (vertex ids offset by voff[g]); the
// degree orientation, the CSR and its weight-sorted row copies are those of the single-graph
// path, since a triangle never spans two graphs and orientation only compares endpoints of
// one edge.  On top of it every graph gets a weight-ordered segment of its entries, grouped
// by 256 coarse weight bins (heaviest first) with the bin offsets kept per graph.
//
// Query.  The threshold descent of the single-graph path runs for all graphs at once: pass i
// gives graph g the band [L_{g,i}, L_{g,i-1}) with L_{g,i} = key(t, t, t), t = the weight of
// the k*G^i-th heaviest edge of g, and streams only the prefix of g's segment whose weights can
// still reach the band (weight floor of Sec. 3.2 with g's largest weight).  A graph drops out
// as soon as it holds >= k triangles (the argument of Sec. 3.2: its top k are among them).
// Triangles go to a region of R records per graph.  A graph whose region overflows is redone
// above the k-th best full key it holds (a valid lower bound), outside the captured sequence.
// The per-graph top-k is taken by rank counting in LDS.  The whole sequence (plan, scan,
// filter, intersect per pass; selection) is captured once per (k, p, launch configuration)
// into a hipGraph and replayed; an autotuner picks the configuration by timing replays.
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "common.h"
#include "enum.h"

namespace {

constexpr uint32_t NB = WBINS / 8; // coarse weight bins per graph
__host__ __device__ inline uint32_t coarse_bin(uint32_t w) { return weight_bin(w) >> 3; }
constexpr uint32_t OVERFLOWED = 0xFFFFFFFFu;
constexpr int ST_HAS_PREV = 1, ST_EXHAUSTED = 2;

struct BState {
    u128 Lprev;
    uint32_t flags;
};

// ----------------------------------------------------------------------------- load kernels
// Local ids -> union ids; flags ids >= n_g (lowest bad graph in bad[1]).
__global__ __launch_bounds__(256) void k_globalize(uint32_t *src, uint32_t *dst, uint64_t m, const uint64_t *eoff,
                                                   const uint64_t *voff, uint32_t count, uint32_t *bad) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = count; // last g with eoff[g] <= e
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (eoff[mid] <= e) lo = mid; else hi = mid;
        }
        while (eoff[lo + 1] <= e) lo++; // skip graphs without edges
        const uint64_t n = voff[lo + 1] - voff[lo];
        const uint32_t s = src[e], d = dst[e];
        if (s >= n || d >= n) {
            atomicOr(&bad[0], 1u);
            atomicMin(&bad[1], lo);
        } else {
            src[e] = (uint32_t)(voff[lo] + s);
            dst[e] = (uint32_t)(voff[lo] + d);
        }
    }
}

// One block per graph: entries per coarse bin (bucket g*NB + NB-1-bin) and the largest weight.
__global__ __launch_bounds__(256) void k_bcount(const uint64_t *voff, const uint64_t *rstart, const uint32_t *rlen,
                                                const uint32_t *wgt, uint32_t *bcnt, uint32_t *gwmax) {
    __shared__ uint32_t h[NB];
    __shared__ uint32_t wmax;
    const uint32_t g = blockIdx.x;
    for (uint32_t t = threadIdx.x; t < NB; t += blockDim.x) h[t] = 0;
    if (threadIdx.x == 0) wmax = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    uint32_t mx = 0;
    for (uint64_t v = voff[g] + (threadIdx.x >> 6); v < voff[g + 1]; v += blockDim.x >> 6) {
        const uint64_t b = rstart[v];
        const uint32_t len = rlen[v];
        for (uint32_t t = lane; t < len; t += 64) {
            const uint32_t w = wgt[b + t];
            mx = w > mx ? w : mx;
            atomicAdd(&h[NB - 1 - coarse_bin(w)], 1u);
        }
    }
    mx = wave_max(mx);
    if (lane == 0) atomicMax(&wmax, mx);
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < NB; t += blockDim.x) bcnt[(uint64_t)g * NB + t] = h[t];
    if (threadIdx.x == 0) gwmax[g] = wmax;
}

// One block per graph: scatter the graph's entries into its weight-ordered segment.
__global__ __launch_bounds__(256) void k_bscatter(const uint64_t *voff, const uint64_t *rstart, const uint32_t *rlen,
                                                  const uint32_t *col, const uint32_t *wgt, const uint64_t *boff,
                                                  uint32_t *bs_src, uint32_t *bs_col, uint32_t *bs_wgt) {
    __shared__ uint32_t cur[NB];
    const uint32_t g = blockIdx.x;
    for (uint32_t t = threadIdx.x; t < NB; t += blockDim.x) cur[t] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (uint64_t v = voff[g] + (threadIdx.x >> 6); v < voff[g + 1]; v += blockDim.x >> 6) {
        const uint64_t b = rstart[v];
        const uint32_t len = rlen[v];
        for (uint32_t t = lane; t < len; t += 64) {
            const uint32_t w = wgt[b + t];
            const uint32_t j = NB - 1 - coarse_bin(w);
            const uint64_t d = boff[(uint64_t)g * NB + j] + atomicAdd(&cur[j], 1u);
            bs_src[d] = (uint32_t)v;
            bs_col[d] = col[b + t];
            bs_wgt[d] = w;
        }
    }
}

// ----------------------------------------------------------------------------- query kernels
// Pass `pass` of the descent, one thread per graph: the graph's band and how many entries of
// its segment to stream (0 once it holds >= k triangles or has had its exhaustive band).
__global__ __launch_bounds__(256) void k_bplan(uint32_t pass, uint32_t count, uint32_t k, int mode, double p,
                                               unsigned long long M, const uint64_t *boff, const uint64_t *gm,
                                               const uint32_t *gwmax, unsigned long long *gcount, BState *st,
                                               Band *bands, uint32_t *Eg) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= count) return;
    BState S;
    if (pass == 0) {
        S.Lprev = 0;
        S.flags = 0;
        gcount[g] = 0;
    } else {
        S = st[g];
    }
    uint32_t E = 0;
    if (gcount[g] < k && !(S.flags & ST_EXHAUSTED)) {
        const uint64_t *bo = boff + (uint64_t)g * NB;
        u128 L = 0;
        if (M < gm[g]) {
            uint32_t lo = 0, hi = NB - 1; // first bucket j with (entries in buckets 0..j) >= M
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (bo[mid + 1] - bo[0] >= M) hi = mid; else lo = mid + 1;
            }
            const uint32_t t = weight_bin_low((NB - 1 - lo) << 3);
            if (t > 1) L = key_of_uniform(mode, t);
        }
        const bool has_prev = S.flags & ST_HAS_PREV;
        if (!has_prev || L < S.Lprev) {
            Band B;
            B.L = L;
            B.Li = B.Lj = B.Ll = 0xFFFFFFFFu;
            B.U = S.Lprev;
            B.hasU = has_prev ? 1 : 0;
            B.mode = mode;
            B.p = p;
            B.theta = mode == MODE_GEN ? key_as_double(L) : 0.0;
            bands[g] = B;
            const uint64_t z = weight_floor(mode, p, L, gwmax[g]);
            if (z == 0) E = (uint32_t)(bo[NB] - bo[0]);
            else if (z <= 0xFFFFFFFFull) E = (uint32_t)(bo[NB - coarse_bin((uint32_t)z)] - bo[0]);
            S.Lprev = L;
            S.flags |= ST_HAS_PREV | (L == 0 ? ST_EXHAUSTED : 0);
        }
    }
    Eg[g] = E;
    st[g] = S;
}

// Restart of the listed graphs above the k-th best full key they hold (kth[g]); every other
// graph streams nothing.
__global__ __launch_bounds__(256) void k_brestart(uint32_t count, const uint8_t *redo, const trec *kth, int mode,
                                                  double p, const uint64_t *boff, const uint32_t *gwmax,
                                                  unsigned long long *gcount, Band *bands, uint32_t *Eg) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= count) return;
    uint32_t E = 0;
    if (redo[g]) {
        const trec r = kth[g];
        Band B;
        B.L = ((u128)r.khi << 64) | r.klo;
        B.Li = r.i;
        B.Lj = r.j;
        B.Ll = r.l;
        B.U = 0;
        B.hasU = 0;
        B.mode = mode;
        B.p = p;
        B.theta = mode == MODE_GEN ? key_as_double(B.L) : 0.0;
        bands[g] = B;
        gcount[g] = 0;
        const uint64_t *bo = boff + (uint64_t)g * NB;
        const uint64_t z = weight_floor(mode, p, B.L, gwmax[g]);
        if (z == 0) E = (uint32_t)(bo[NB] - bo[0]);
        else if (z <= 0xFFFFFFFFull) E = (uint32_t)(bo[NB - coarse_bin((uint32_t)z)] - bo[0]);
    }
    Eg[g] = E;
}

// Exclusive prefix of Eg[0..count) into poff[0..count] (one block; count is a few thousand).
__global__ __launch_bounds__(1024) void k_bscan(const uint32_t *Eg, uint32_t count, uint64_t *poff) {
    __shared__ uint64_t wsum[16];
    const uint32_t per = (count + 1023) / 1024;
    const uint32_t lo = threadIdx.x * per, hi = lo + per < count ? lo + per : count;
    uint64_t sum = 0;
    for (uint32_t t = lo; t < hi; t++) sum += Eg[t];
    const uint64_t incl = wave_incl_scan(sum);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint64_t run = incl - sum;
    for (int w = 0; w < wv; w++) run += wsum[w];
    for (uint32_t t = lo; t < hi; t++) {
        poff[t] = run;
        run += Eg[t];
    }
    if (threadIdx.x == 1023) poff[count] = run;
}

constexpr uint32_t SEL_TILE = 1024;

// Per-graph top-k by rank counting: a record's rank is the number of records of its graph
// that are better under (key desc, i, j, l asc).  Writes the first min(k, N) triangles with
// local ids, or marks the graph OVERFLOWED when its region overflowed.  With `kth` set, the
// listed (overflowed) graphs instead report their record of rank k-1 among the R kept.
__global__ __launch_bounds__(256) void k_bselect(const trec *rec, uint32_t R, const unsigned long long *gcount,
                                                 const uint8_t *only, uint32_t count, uint32_t k, int mode,
                                                 const uint64_t *voff, tt_triangle *out, uint32_t *n_out, trec *kth) {
    __shared__ trec tile[SEL_TILE];
    for (uint32_t g = blockIdx.x; g < count; g += gridDim.x) {
        if (only && !only[g]) continue;
        const unsigned long long cnt = gcount[g];
        if (!kth && cnt > R) {
            if (threadIdx.x == 0) n_out[g] = OVERFLOWED;
            continue;
        }
        const uint32_t N = (uint32_t)(cnt < R ? cnt : R);
        const uint32_t K = N < k ? N : k;
        const trec *base = rec + (uint64_t)g * R;
        const uint32_t off = (uint32_t)voff[g];
        for (uint32_t r0 = 0; r0 < N; r0 += blockDim.x) {
            const uint32_t idx = r0 + threadIdx.x;
            const bool has = idx < N;
            trec me;
            if (has) me = base[idx];
            uint32_t rank = 0;
            for (uint32_t t0 = 0; t0 < N; t0 += SEL_TILE) {
                const uint32_t cover = N - t0 < SEL_TILE ? N - t0 : SEL_TILE;
                __syncthreads();
                for (uint32_t t = threadIdx.x; t < cover; t += blockDim.x) tile[t] = base[t0 + t];
                __syncthreads();
                if (has)
                    for (uint32_t t = 0; t < cover; t++) rank += better(tile[t], me) ? 1u : 0u;
            }
            if (has && rank < K) {
                if (kth) {
                    if (rank == K - 1) kth[g] = me;
                } else {
                    tt_triangle o;
                    o.i = me.i - off;
                    o.j = me.j - off;
                    o.l = me.l - off;
                    o._pad = 0;
                    o.score = key_to_score(mode, ((u128)me.khi << 64) | me.klo);
                    out[(uint64_t)g * k + rank] = o;
                }
            }
        }
        if (!kth && threadIdx.x == 0) n_out[g] = K;
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------- host side
struct BatchCfg {
    uint32_t growth;        // rank ratio between consecutive bands
    uint32_t filter_mul;    // filter blocks per CU
    uint32_t inter_mul;     // intersect blocks per CU
};
const BatchCfg CONFIGS[] = {
    {4, 4, 4},  {4, 4, 8},  {4, 4, 16},  {4, 16, 4},  {4, 16, 8},  {4, 16, 16},
    {16, 4, 4}, {16, 4, 8}, {16, 4, 16}, {16, 16, 4}, {16, 16, 8}, {16, 16, 16},
};
constexpr int NCONFIGS = (int)(sizeof(CONFIGS) / sizeof(CONFIGS[0]));

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

} // namespace

struct tt_batch {
    tt_graph *g = nullptr; // the disjoint union
    uint32_t count = 0;
    uint64_t max_m = 0;
    std::vector<uint64_t> voff_h;
    uint64_t *voff = nullptr; // [count+1]
    uint64_t *gm = nullptr;   // [count] edges per graph
    uint32_t *gwmax = nullptr;
    uint64_t *boff = nullptr; // [count*NB+1]
    uint64_t *goff = nullptr; // [count+1] start of graph g's segment (= boff[g*NB])
    uint32_t *bs_src = nullptr, *bs_col = nullptr, *bs_wgt = nullptr;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    // query state (sized for the largest k seen)
    uint32_t R = 0, kcap = 0;
    Band *bands = nullptr;
    BState *st = nullptr;
    uint32_t *Eg = nullptr;
    uint64_t *poff = nullptr;
    unsigned long long *gcount = nullptr;
    trec *rec = nullptr, *kth = nullptr;
    cand *C = nullptr;
    uint32_t *ccnt = nullptr;
    unsigned long long *spart = nullptr, *dstat = nullptr;
    tt_triangle *dout = nullptr;
    uint32_t *dn = nullptr;
    uint8_t *redo = nullptr;
    unsigned long long extra[5] = {}; // counters of the restart passes of the latest query
    hipEvent_t ev[2] = {};
    struct Plan {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        uint32_t passes = 0;
    };
    std::map<std::tuple<uint32_t, uint64_t, int>, Plan> plans; // (k, bits of p, config)
    std::map<std::pair<uint32_t, uint64_t>, int> tuned;        // (k, bits of p) -> config
    std::mutex mu;
};

namespace {

uint64_t p_bits(double p) {
    uint64_t b;
    std::memcpy(&b, &p, 8);
    return b;
}

void free_query_state(tt_batch *b) {
    void *ptrs[] = {b->bands, b->st, b->Eg, b->poff, b->gcount, b->rec, b->kth, b->C, b->ccnt,
                    b->spart, b->dstat, b->dout, b->dn, b->redo};
    for (void *p : ptrs) dev_free(nullptr, p, 0);
    b->bands = nullptr; b->st = nullptr; b->Eg = nullptr; b->poff = nullptr; b->gcount = nullptr;
    b->rec = b->kth = nullptr; b->C = nullptr; b->ccnt = nullptr; b->spart = b->dstat = nullptr;
    b->dout = nullptr; b->dn = nullptr; b->redo = nullptr;
    b->R = b->kcap = 0;
}

void drop_plans(tt_batch *b) {
    for (auto &kv : b->plans) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    b->plans.clear();
}

// Query buffers for top-k with k <= kcap (captured plans hold their addresses, so they are
// dropped whenever the buffers move).
int ensure_query_state(tt_batch *b, uint32_t k) {
    if (b->kcap >= k && b->bands) return TT_OK;
    drop_plans(b);
    free_query_state(b);
    const uint64_t n = b->count, m = b->g->m;
    const uint32_t R = std::max<uint32_t>(2048, 16 * k);
    int rc;
    if ((rc = dev_alloc(nullptr, (void **)&b->bands, n * sizeof(Band))) ||
        (rc = dev_alloc(nullptr, (void **)&b->st, n * sizeof(BState))) ||
        (rc = dev_alloc(nullptr, (void **)&b->Eg, (n + 1) * 4)) ||
        (rc = dev_alloc(nullptr, (void **)&b->poff, (n + 1) * 8)) ||
        (rc = dev_alloc(nullptr, (void **)&b->gcount, n * 8)) ||
        (rc = dev_alloc(nullptr, (void **)&b->rec, n * R * sizeof(trec))) ||
        (rc = dev_alloc(nullptr, (void **)&b->kth, n * sizeof(trec))) ||
        (rc = dev_alloc(nullptr, (void **)&b->C, (m + 1) * sizeof(cand))) ||
        (rc = dev_alloc(nullptr, (void **)&b->ccnt, MAX_SEG * 4)) ||
        (rc = dev_alloc(nullptr, (void **)&b->spart, 5 * STAT_SLOTS * 8)) ||
        (rc = dev_alloc(nullptr, (void **)&b->dstat, 16 * 8)) ||
        (rc = dev_alloc(nullptr, (void **)&b->dout, n * k * sizeof(tt_triangle) + 8)) ||
        (rc = dev_alloc(nullptr, (void **)&b->dn, n * 4)) ||
        (rc = dev_alloc(nullptr, (void **)&b->redo, n + 1))) {
        free_query_state(b);
        return rc;
    }
    HIP_TRY(hipMemsetAsync(b->spart, 0, 5 * STAT_SLOTS * 8, b->stream));
    HIP_TRY(hipMemsetAsync(b->ccnt, 0, MAX_SEG * 4, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->R = R;
    b->kcap = k;
    return TT_OK;
}

uint32_t passes_for(const tt_batch *b, uint32_t k, uint32_t growth) {
    uint32_t P = 1;
    for (unsigned long long M = k; M < b->max_m && P < 40; M *= growth) P++;
    return P;
}

EnumArgs batch_args(const tt_batch *b, uint32_t k, double p, const BatchCfg &c) {
    const tt_graph *g = b->g;
    EnumArgs A;
    std::memset(&A, 0, sizeof(A));
    A.rstart = g->rstart;
    A.rlen = g->rlen;
    A.col = g->col;
    A.wgt = g->wgt;
    A.wcol = g->wcol;
    A.wwgt = g->wwgt;
    A.wpos = g->wpos;
    A.maxw = g->maxw;
    A.s_src = b->bs_src;
    A.s_col = b->bs_col;
    A.s_wgt = b->bs_wgt;
    A.B.mode = mode_of(p);
    A.B.p = p;
    A.out = b->rec;
    A.stats = b->spart;
    A.C = b->C;
    A.ccnt = b->ccnt;
    A.nseg = std::min<uint32_t>((uint32_t)num_cus() * c.filter_mul, MAX_SEG);
    A.bands = b->bands;
    A.poff = b->poff;
    A.goff = b->boff; // graph g's segment starts at bucket g*NB: goff[g] = boff[g*NB] (stride NB)
    A.ng = b->count;
    A.gcount = b->gcount;
    A.R = b->R;
    (void)k;
    return A;
}

// The stream offsets are boff[g*NB]; the kernels index goff[g], so a strided copy is kept.
__global__ void k_goff(const uint64_t *boff, uint32_t count, uint64_t *goff) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < count) goff[g] = boff[(uint64_t)g * NB];
}

int enqueue_pass(tt_batch *b, const EnumArgs &A, const BatchCfg &c) {
    hipStream_t s = b->stream;
    k_bscan<<<1, 1024, 0, s>>>(b->Eg, b->count, b->poff);
    k_filter<FILTER_NONE, true><<<A.nseg, 256, 0, s>>>(A);
    k_intersect<FILTER_NONE, true><<<(unsigned)num_cus() * c.inter_mul, 256, 0, s>>>(A);
    HIP_TRY(hipGetLastError());
    return TT_OK;
}

// The launch sequence of one query: every pass of the descent, then the per-graph selection
// and the counters.  Nothing in it allocates, copies or sets memory, so it can be captured.
int enqueue_query(tt_batch *b, uint32_t k, double p, const BatchCfg &c, const uint64_t *goff) {
    hipStream_t s = b->stream;
    const int mode = mode_of(p);
    EnumArgs A = batch_args(b, k, p, c);
    A.goff = goff;
    const uint32_t P = passes_for(b, k, c.growth);
    const unsigned pg = (b->count + 255) / 256;
    unsigned long long M = k;
    for (uint32_t i = 0; i < P; i++) {
        const unsigned long long Mi = i + 1 == P ? ~0ull : M; // the last band is exhaustive
        k_bplan<<<pg, 256, 0, s>>>(i, b->count, k, mode, p, Mi, b->boff, b->gm, b->gwmax, b->gcount, b->st,
                                   b->bands, b->Eg);
        int rc = enqueue_pass(b, A, c);
        if (rc) return rc;
        M = M > (~0ull / c.growth) ? ~0ull : M * c.growth;
    }
    const unsigned sg = std::min<unsigned>(b->count, (unsigned)num_cus() * 8);
    k_bselect<<<sg, 256, 0, s>>>(b->rec, b->R, b->gcount, nullptr, b->count, k, mode, b->voff, b->dout, b->dn,
                                 nullptr);
    k_reduce_stats<<<5, 256, 0, s>>>(b->spart, b->dstat);
    HIP_TRY(hipGetLastError());
    return TT_OK;
}

} // namespace

// ----------------------------------------------------------------------------- C ABI
namespace {

int batch_load_common(uint32_t count, const uint32_t *n, const uint64_t *m, const uint32_t *src, const uint32_t *dst,
                      const uint32_t *w, void *stream, bool host, tt_batch **out) {
    if (!out) return fail(TT_E_ARG, "out is NULL");
    *out = nullptr;
    if (count && (!n || !m)) return fail(TT_E_ARG, "n or m is NULL");
    std::vector<uint64_t> voff(count + 1, 0), eoff(count + 1, 0);
    uint64_t max_m = 0;
    for (uint32_t g = 0; g < count; g++) {
        voff[g + 1] = voff[g] + n[g];
        eoff[g + 1] = eoff[g] + m[g];
        max_m = std::max<uint64_t>(max_m, m[g]);
    }
    const uint64_t N = voff[count], M = eoff[count];
    if (N > 0xFFFFFFFEull) return fail(TT_E_TOO_LARGE, "the graphs hold more than 2^32 - 2 vertices together");
    if (M > 0xFFFFFFFEull) return fail(TT_E_TOO_LARGE, "the graphs hold more than 2^32 - 2 edges together");
    if (M && (!src || !dst || !w)) return fail(TT_E_ARG, "src, dst or w is NULL");
    tt_batch *b = new (std::nothrow) tt_batch();
    if (!b) return fail(TT_E_NOMEM, "host allocation failed");
    b->count = count;
    b->max_m = max_m;
    b->voff_h = voff;
    // queries run on a stream of the batch's own (it is captured); loading runs on the
    // caller's stream when one is given, after the work that produced the inputs
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return fail(TT_E_DEVICE, "hipStreamCreate failed");
    }
    b->owns_stream = true;
    hipStream_t s = stream ? (hipStream_t)stream : b->stream;
    if (!host && !stream && hipStreamSynchronize(nullptr) != hipSuccess) {
        batch_free(b);
        return fail(TT_E_DEVICE, "hipStreamSynchronize failed");
    }
    uint32_t *us = nullptr, *bad = nullptr;
    uint64_t *eoff_d = nullptr;
    auto body = [&]() -> int {
        int rc;
        if ((rc = dev_alloc(nullptr, (void **)&us, 3 * M * 4 + 4)) ||
            (rc = dev_alloc(nullptr, (void **)&eoff_d, (count + 1) * 8)) ||
            (rc = dev_alloc(nullptr, (void **)&bad, 8)) ||
            (rc = dev_alloc(nullptr, (void **)&b->voff, (count + 1) * 8)) ||
            (rc = dev_alloc(nullptr, (void **)&b->gm, (count + 1) * 8)) ||
            (rc = dev_alloc(nullptr, (void **)&b->gwmax, (count + 1) * 4)))
            return rc;
        const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        if (M) {
            HIP_TRY(hipMemcpyAsync(us, src, M * 4, kind, s));
            HIP_TRY(hipMemcpyAsync(us + M, dst, M * 4, kind, s));
            HIP_TRY(hipMemcpyAsync(us + 2 * M, w, M * 4, kind, s));
        }
        HIP_TRY(hipMemcpyAsync(eoff_d, eoff.data(), (count + 1) * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->voff, voff.data(), (count + 1) * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(b->gm, m, (uint64_t)count * 8, hipMemcpyHostToDevice, s));
        const uint32_t init[2] = {0, 0xFFFFFFFFu};
        HIP_TRY(hipMemcpyAsync(bad, init, 8, hipMemcpyHostToDevice, s));
        if (M) {
            const unsigned grid = (unsigned)std::min<uint64_t>((M + 255) / 256, (uint64_t)num_cus() * 16);
            k_globalize<<<grid, 256, 0, s>>>(us, us + M, M, eoff_d, b->voff, count, bad);
            HIP_TRY(hipGetLastError());
        }
        uint32_t hb[2];
        HIP_TRY(hipMemcpyAsync(hb, bad, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hb[0]) return fail(TT_E_VERTEX_RANGE, "graph " + std::to_string(hb[1]) + ": vertex id >= its n");
        if ((rc = graph_load_device((uint32_t)N, M, us, us + M, us + 2 * M, s, &b->g))) return rc;
        // per-graph weight-ordered segments
        const uint64_t nb = (uint64_t)count * NB + 1;
        uint32_t *bcnt = nullptr;
        if ((rc = dev_alloc(nullptr, (void **)&bcnt, nb * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&b->boff, nb * 8)) ||
            (rc = dev_alloc(nullptr, (void **)&b->goff, ((uint64_t)count + 1) * 8)) ||
            (rc = dev_alloc(nullptr, (void **)&b->bs_src, (M + 1) * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&b->bs_col, (M + 1) * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&b->bs_wgt, (M + 1) * 4))) {
            dev_free(nullptr, bcnt, 0);
            return rc;
        }
        HIP_TRY(hipMemsetAsync(bcnt, 0, nb * 4, s));
        if (count) {
            k_bcount<<<count, 256, 0, s>>>(b->voff, b->g->rstart, b->g->rlen, b->g->wgt, bcnt, b->gwmax);
            HIP_TRY(hipGetLastError());
        }
        rc = exclusive_scan_u32_to_u64(bcnt, b->boff, nb, s, nullptr);
        if (!rc && count) {
            k_bscatter<<<count, 256, 0, s>>>(b->voff, b->g->rstart, b->g->rlen, b->g->col, b->g->wgt, b->boff,
                                             b->bs_src, b->bs_col, b->bs_wgt);
            HIP_TRY(hipGetLastError());
        }
        if (!rc && count) {
            HIP_TRY(hipMemsetAsync(b->goff, 0, ((uint64_t)count + 1) * 8, s));
            k_goff<<<(count + 255) / 256, 256, 0, s>>>(b->boff, count, b->goff);
            HIP_TRY(hipGetLastError());
        }
        (void)hipStreamSynchronize(s);
        dev_free(nullptr, bcnt, 0);
        if (rc) return rc;
        HIP_TRY(hipEventCreate(&b->ev[0]));
        HIP_TRY(hipEventCreate(&b->ev[1]));
        return TT_OK;
    };
    int rc = body();
    (void)hipStreamSynchronize(s);
    dev_free(nullptr, us, 0);
    dev_free(nullptr, eoff_d, 0);
    dev_free(nullptr, bad, 0);
    if (rc) {
        batch_free(b);
        return rc;
    }
    *out = b;
    set_error("");
    return TT_OK;
}

// Runs one query with configuration c: replays (or first captures) its plan, or enqueues it
// directly when `eager`; then redoes overflowed graphs.  Results stay in b->dout / b->dn.
int run_batch(tt_batch *b, uint32_t k, double p, int ci, bool eager, uint32_t *restarts, double *ms) {
    const BatchCfg &c = CONFIGS[ci];
    hipStream_t s = b->stream;
    uint64_t *goff = b->goff;
    int rc;
    HIP_TRY(hipEventRecord(b->ev[0], s));
    if (eager) {
        if ((rc = enqueue_query(b, k, p, c, goff))) return rc;
    } else {
        auto key = std::make_tuple(k, p_bits(p), ci);
        auto it = b->plans.find(key);
        if (it == b->plans.end()) {
            tt_batch::Plan pl;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            rc = enqueue_query(b, k, p, c, goff);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (e != hipSuccess) return fail(TT_E_DEVICE, std::string("stream capture: ") + hipGetErrorString(e));
            pl.graph = graph;
            HIP_TRY(hipGraphInstantiate(&pl.exec, graph, nullptr, nullptr, 0));
            pl.passes = passes_for(b, k, c.growth);
            it = b->plans.emplace(key, pl).first;
        }
        HIP_TRY(hipGraphLaunch(it->second.exec, s));
    }
    HIP_TRY(hipEventRecord(b->ev[1], s));
    std::vector<uint32_t> hn(b->count);
    std::memset(b->extra, 0, sizeof(b->extra));
    HIP_TRY(hipMemcpyAsync(hn.data(), b->dn, (uint64_t)b->count * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ms) {
        float f = 0.f;
        (void)hipEventElapsedTime(&f, b->ev[0], b->ev[1]);
        *ms = f;
    }
    // graphs whose region overflowed: redo above the k-th best key they hold
    const int mode = mode_of(p);
    EnumArgs A = batch_args(b, k, p, c);
    A.goff = goff;
    const unsigned pg = (b->count + 255) / 256;
    for (int round = 0; round < 64; round++) {
        std::vector<uint8_t> redo(b->count + 1, 0);
        uint32_t nredo = 0;
        for (uint32_t g = 0; g < b->count; g++)
            if (hn[g] == OVERFLOWED) { redo[g] = 1; nredo++; }
        if (!nredo) return TT_OK;
        if (restarts) *restarts += nredo;
        HIP_TRY(hipMemcpyAsync(b->redo, redo.data(), b->count + 1, hipMemcpyHostToDevice, s));
        const unsigned sg = std::min<unsigned>(b->count, (unsigned)num_cus() * 8);
        k_bselect<<<sg, 256, 0, s>>>(b->rec, b->R, b->gcount, b->redo, b->count, k, mode, b->voff, nullptr, nullptr,
                                     b->kth);
        k_brestart<<<pg, 256, 0, s>>>(b->count, b->redo, b->kth, mode, p, b->boff, b->gwmax, b->gcount, b->bands,
                                      b->Eg);
        if ((rc = enqueue_pass(b, A, c))) return rc;
        k_bselect<<<sg, 256, 0, s>>>(b->rec, b->R, b->gcount, b->redo, b->count, k, mode, b->voff, b->dout, b->dn,
                                     nullptr);
        k_reduce_stats<<<5, 256, 0, s>>>(b->spart, b->dstat + 8);
        HIP_TRY(hipGetLastError());
        unsigned long long st[5];
        HIP_TRY(hipMemcpyAsync(hn.data(), b->dn, (uint64_t)b->count * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(st, b->dstat + 8, sizeof(st), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int c2 = 0; c2 < 5; c2++) b->extra[c2] += st[c2];
    }
    return fail(TT_E_DEVICE, "batched query: overflow restarts did not converge");
}

int autotune(tt_batch *b, uint32_t k, double p, int *best, double *tune_ms) {
    const double t0 = now_ms();
    double best_ms = 1e300;
    int bi = 0;
    for (int ci = 0; ci < NCONFIGS; ci++) {
        double ms = 0, tot = 0;
        int rc = run_batch(b, k, p, ci, false, nullptr, &ms); // capture + warm-up
        if (rc) return rc;
        for (int r = 0; r < 3; r++) {
            if ((rc = run_batch(b, k, p, ci, false, nullptr, &ms))) return rc;
            tot += ms;
        }
        if (tot < best_ms) { best_ms = tot; bi = ci; }
    }
    // plans that lost are released
    for (auto it = b->plans.begin(); it != b->plans.end();) {
        if (std::get<0>(it->first) == k && std::get<1>(it->first) == p_bits(p) && std::get<2>(it->first) != bi) {
            (void)hipGraphExecDestroy(it->second.exec);
            (void)hipGraphDestroy(it->second.graph);
            it = b->plans.erase(it);
        } else {
            ++it;
        }
    }
    *best = bi;
    if (tune_ms) *tune_ms = now_ms() - t0;
    return TT_OK;
}

} // namespace

extern "C" int batch_load(uint32_t count, const uint32_t *n, const uint64_t *m, const uint32_t *src,
                          const uint32_t *dst, const uint32_t *w, tt_batch **out) {
    return batch_load_common(count, n, m, src, dst, w, nullptr, true, out);
}

extern "C" int batch_load_device(uint32_t count, const uint32_t *n, const uint64_t *m, const uint32_t *src,
                                 const uint32_t *dst, const uint32_t *w, void *stream, tt_batch **out) {
    return batch_load_common(count, n, m, src, dst, w, stream, false, out);
}

extern "C" uint32_t batch_num_configs(void) { return (uint32_t)NCONFIGS; }

extern "C" uint32_t batch_num_graphs(const tt_batch *b) { return b ? b->count : 0; }

extern "C" int batch_topk_ex(tt_batch *b, uint32_t k, double p, int config, uint32_t flags, tt_triangle *out,
                             uint32_t *n_out, tt_batch_stats *stats) {
    const double t0 = now_ms();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (!b) return fail(TT_E_ARG, "batch is NULL");
    if (!n_out && b->count) return fail(TT_E_ARG, "n_out is NULL");
    for (uint32_t g = 0; g < b->count; g++) n_out[g] = 0;
    if (std::isnan(p)) return fail(TT_E_ARG, "p is NaN");
    if (k && b->count && !out) return fail(TT_E_ARG, "out is NULL");
    if (config < -1 || config >= NCONFIGS) return fail(TT_E_ARG, "config out of range");
    if (flags & ~(uint32_t)TT_BATCH_EAGER) return fail(TT_E_ARG, "unknown flags");
    if (k == 0 || b->count == 0 || b->g->m == 0) { set_error(""); return TT_OK; }
    std::lock_guard<std::mutex> lock(b->mu);
    (void)hipSetDevice(b->g->device);
    int rc = ensure_query_state(b, k);
    if (rc) return rc;
    int ci = config;
    double tune_ms = 0.0;
    if (ci < 0) {
        auto key = std::make_pair(k, p_bits(p));
        auto it = b->tuned.find(key);
        if (it == b->tuned.end()) {
            if ((rc = autotune(b, k, p, &ci, &tune_ms))) return rc;
            b->tuned[key] = ci;
        } else {
            ci = it->second;
        }
    }
    uint32_t restarts = 0;
    double ms = 0.0;
    if ((rc = run_batch(b, k, p, ci, (flags & TT_BATCH_EAGER) != 0, &restarts, &ms))) return rc;
    hipStream_t s = b->stream;
    HIP_TRY(hipMemcpyAsync(n_out, b->dn, (uint64_t)b->count * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(out, b->dout, (uint64_t)b->count * k * sizeof(tt_triangle), hipMemcpyDeviceToHost, s));
    unsigned long long st[5] = {};
    HIP_TRY(hipMemcpyAsync(st, b->dstat, sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (stats) {
        stats->config = (uint32_t)ci;
        stats->growth = CONFIGS[ci].growth;
        stats->filter_blocks = std::min<uint32_t>((uint32_t)num_cus() * CONFIGS[ci].filter_mul, MAX_SEG);
        stats->intersect_blocks = (uint32_t)num_cus() * CONFIGS[ci].inter_mul;
        stats->passes = passes_for(b, k, CONFIGS[ci].growth);
        stats->restarts = restarts;
        stats->candidate_edges = st[0] + b->extra[0];
        stats->intersected_entries = st[1] + b->extra[1];
        stats->triangles_emitted = st[2] + b->extra[2];
        stats->edges_streamed = st[3] + b->extra[3];
        stats->launch_ms = ms;
        stats->tune_ms = tune_ms;
        stats->total_ms = now_ms() - t0;
    }
    set_error("");
    return TT_OK;
}

extern "C" int batch_topk(tt_batch *b, uint32_t k, double p, tt_triangle *out, uint32_t *n_out) {
    return batch_topk_ex(b, k, p, -1, 0, out, n_out, nullptr);
}

extern "C" void batch_free(tt_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_plans(b);
    free_query_state(b);
    void *ptrs[] = {b->voff, b->gm, b->gwmax, b->boff, b->goff, b->bs_src, b->bs_col, b->bs_wgt};
    for (void *p : ptrs) dev_free(nullptr, p, 0);
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->g) graph_free(b->g);
    if (b->owns_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}
