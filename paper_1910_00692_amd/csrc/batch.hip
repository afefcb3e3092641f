// batch.hip — the batched form: one top-k per graph for many independent graphs of uneven
// size (the problem of Sec. 1 solved once per graph), in one captured launch sequence.
//
// Layout.  The graphs are loaded as one disjoint union (vertex ids offset by voff[g]); the
// degree orientation, the CSR and its weight-sorted row copies are those of the single-graph
// path, since a triangle never spans two graphs and orientation only compares endpoints of
// one edge.  For each p queried (the two latest are kept) every graph gets a segment of its
// entries ordered by their bound m_p(w_uv, maxw(u), maxw(v)) (the heaviest triangle an entry
// can be the base of, Sec. 3.2), grouped by 256 coarse bins, highest first, with the bin
// offsets kept per graph.
//
// Query.  The threshold descent of the single-graph path runs for all graphs at once: pass i
// gives graph g the band [L_{g,i}, L_{g,i-1}) with L_{g,i} = key(t, t, t), t = the bound of
// the k*G^i-th entry of g's segment, and streams exactly the prefix of the segment whose
// bounds reach t (no other entry can be the base of a triangle in the band).  A graph drops
// out as soon as it holds >= k triangles (the argument of Sec. 3.2: its top k are among them).
// Triangles go to a region of R records per graph.  A graph whose region overflows is redone
// above the k-th best full key it holds (a valid lower bound), outside the captured sequence.
// The per-graph top-k is taken by block-wide selection rounds (small k) or rank counting.  The whole sequence (plan, scan,
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

// One block per graph: entries per coarse bound bin (bucket g*NB + NB-1-bin).
__global__ __launch_bounds__(256) void k_ocount(const uint64_t *voff, const uint64_t *rstart, const uint32_t *rlen,
                                                const uint32_t *col, const uint32_t *wgt, const uint32_t *maxw,
                                                int mode, double p, uint32_t *bcnt) {
    __shared__ uint32_t h[NB];
    const uint32_t g = blockIdx.x;
    for (uint32_t t = threadIdx.x; t < NB; t += blockDim.x) h[t] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (uint64_t v = voff[g] + (threadIdx.x >> 6); v < voff[g + 1]; v += blockDim.x >> 6) {
        const uint64_t b = rstart[v];
        const uint32_t len = rlen[v], Wu = maxw[v];
        for (uint32_t t = lane; t < len; t += 64) {
            const uint32_t ub = entry_bound(mode, p, wgt[b + t], Wu, maxw[col[b + t]]);
            atomicAdd(&h[NB - 1 - coarse_bin(ub)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < NB; t += blockDim.x) bcnt[(uint64_t)g * NB + t] = h[t];
}

// One block per graph: scatter the graph's entries into its bound-ordered segment.
__global__ __launch_bounds__(256) void k_oscatter(const uint64_t *voff, const uint64_t *rstart, const uint32_t *rlen,
                                                  const uint32_t *col, const uint32_t *wgt, const uint32_t *maxw,
                                                  int mode, double p, const uint64_t *boff, uint32_t *o_src,
                                                  uint32_t *o_col, uint32_t *o_wgt) {
    __shared__ uint32_t cur[NB];
    const uint32_t g = blockIdx.x;
    for (uint32_t t = threadIdx.x; t < NB; t += blockDim.x) cur[t] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (uint64_t v = voff[g] + (threadIdx.x >> 6); v < voff[g + 1]; v += blockDim.x >> 6) {
        const uint64_t b = rstart[v];
        const uint32_t len = rlen[v], Wu = maxw[v];
        for (uint32_t t = lane; t < len; t += 64) {
            const uint32_t c = col[b + t], w = wgt[b + t];
            const uint32_t j = NB - 1 - coarse_bin(entry_bound(mode, p, w, Wu, maxw[c]));
            const uint64_t d = boff[(uint64_t)g * NB + j] + atomicAdd(&cur[j], 1u);
            o_src[d] = (uint32_t)v;
            o_col[d] = c;
            o_wgt[d] = w;
        }
    }
}

// ----------------------------------------------------------------------------- query kernels
// Pass `pass` of the descent, one thread per graph: the graph's band and how many entries of
// its bound-ordered segment to stream (0 once it holds >= k triangles or has had its
// exhaustive band).
__global__ __launch_bounds__(256) void k_bplan(uint32_t pass, uint32_t count, uint32_t k, int mode, double p,
                                               unsigned long long M, const uint64_t *boff,
                                               unsigned long long *gcount, BState *st, Band *bands, uint32_t *Eg) {
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
        const uint64_t all = bo[NB] - bo[0];
        u128 L = 0;
        uint64_t En = all;
        if (M < all) {
            uint32_t lo = 0, hi = NB - 1; // first bucket j with (entries in buckets 0..j) >= M
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (bo[mid + 1] - bo[0] >= M) hi = mid; else lo = mid + 1;
            }
            // every triangle scoring >= t has its base entry's bound >= t, in buckets 0..lo
            const uint32_t t = weight_bin_low((NB - 1 - lo) << 3);
            if (t > 1) {
                L = key_of_uniform(mode, t);
                En = bo[lo + 1] - bo[0];
            }
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
            E = (uint32_t)En;
            S.Lprev = L;
            S.flags |= ST_HAS_PREV | (L == 0 ? ST_EXHAUSTED : 0);
        }
    }
    Eg[g] = E;
    st[g] = S;
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
constexpr uint32_t SEL_ROUNDS = 32; // up to this k, the thresholded selection
constexpr uint32_t SEL_REG = 8;     // records per thread held in registers by it

__device__ __forceinline__ void put_result(const trec &me, uint32_t off, int mode, tt_triangle *dst) {
    tt_triangle o;
    o.i = me.i - off;
    o.j = me.j - off;
    o.l = me.l - off;
    o._pad = 0;
    o.score = key_to_score(mode, ((u128)me.khi << 64) | me.klo);
    *dst = o;
}

// Lane src's record, broadcast to the whole wave (src is wave-uniform).
__device__ __forceinline__ trec readlane_rec(const trec &r, int src) {
    trec o;
    o.khi = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(r.khi >> 32), src) << 32) |
            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)r.khi, src);
    o.klo = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(r.klo >> 32), src) << 32) |
            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)r.klo, src);
    o.i = (uint32_t)__builtin_amdgcn_readlane((int)r.i, src);
    o.j = (uint32_t)__builtin_amdgcn_readlane((int)r.j, src);
    o.l = (uint32_t)__builtin_amdgcn_readlane((int)r.l, src);
    o.pad = 0;
    return o;
}

// Rank of each lane's `me` among the `v` of the lanes in `mask` (records better than it).
__device__ __forceinline__ uint32_t wave_rank(const trec &me, const trec &v, uint64_t mask) {
    uint32_t rank = 0;
    while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        rank += better(readlane_rec(v, src), me) ? 1u : 0u;
    }
    return rank;
}

constexpr uint32_t WSEL_MAX = 64 * SEL_REG; // records a wave selects from

// The best K (<= SEL_ROUNDS) of N (<= WSEL_MAX) records at `base`, by one wave, in registers
// only.  N <= 64: every lane holds one record and ranks it against the others.  Otherwise the
// K-th best of the 64 lane bests is a lower bound on the K-th best record, at most SEL_REG*K
// records reach it, and only those are ranked.  Rank r goes to out[r] (ids minus off).
__device__ __forceinline__ void wave_topk(const trec *base, uint32_t N, uint32_t K, uint32_t off, int mode,
                                          tt_triangle *out) {
    const uint32_t lane = threadIdx.x & 63;
    if (N <= 64) {
        const bool has = lane < N;
        const trec me = has ? base[lane] : worst_rec();
        const uint32_t rank = wave_rank(me, me, __ballot(has));
        if (has && rank < K) put_result(me, off, mode, out + rank);
        return;
    }
    trec loc[SEL_REG];
    trec lb = worst_rec();
#pragma unroll
    for (uint32_t q = 0; q < SEL_REG; q++) {
        const uint32_t idx = lane + q * 64;
        loc[q] = idx < N ? base[idx] : worst_rec();
        if (better(loc[q], lb)) lb = loc[q];
    }
    // every lane holds a record (N > 64); the lane best of rank K-1 is the bound
    const uint32_t rb = wave_rank(lb, lb, ~0ull);
    const int xl = __ffsll((unsigned long long)__ballot(rb == K - 1)) - 1;
    const trec x = readlane_rec(lb, xl);
    bool keep[SEL_REG];
    uint32_t rank[SEL_REG];
#pragma unroll
    for (uint32_t q = 0; q < SEL_REG; q++) {
        keep[q] = lane + q * 64 < N && !better(x, loc[q]);
        rank[q] = 0;
    }
#pragma unroll
    for (uint32_t q2 = 0; q2 < SEL_REG; q2++) {
        uint64_t m = __ballot(keep[q2]);
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const trec o = readlane_rec(loc[q2], src);
#pragma unroll
            for (uint32_t q = 0; q < SEL_REG; q++) rank[q] += better(o, loc[q]) ? 1u : 0u;
        }
    }
#pragma unroll
    for (uint32_t q = 0; q < SEL_REG; q++)
        if (keep[q] && rank[q] < K) put_result(loc[q], off, mode, out + rank[q]);
}

union SelShared {
    struct {
        trec wtop[4][SEL_ROUNDS];        // each wave's best K per-thread bests
        trec cand[SEL_REG * SEL_ROUNDS]; // records at or above the threshold
        trec x;
        uint32_t ccount;
    } small;
    trec tile[SEL_TILE];
};

// The best K of the N records at `base` under (key desc, i, j, l asc), by one block of 256
// threads.  Small K with N <= 256*SEL_REG: every thread holds its records in registers; the
// K-th best of the 256 per-thread bests (found from each wave's best K) is a lower bound on
// the K-th best record (K real records reach it), and at most SEL_REG*K records reach that
// bound (only threads whose best does), so ranks are counted among those alone.  Otherwise
// rank counting over all N records.  Rank r goes to out[r] (local ids, ids minus off) if out
// is set; the record of rank K-1 to *kth if kth is set.
__device__ __forceinline__ void block_topk(const trec *base, uint32_t N, uint32_t K, uint32_t off, int mode,
                                           tt_triangle *out, trec *kth, SelShared &sh) {
    const uint32_t tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    if (K == 0) return;
    if (K <= SEL_ROUNDS && N <= SEL_REG * 256) {
        trec loc[SEL_REG];
        trec v = worst_rec();
#pragma unroll
        for (uint32_t q = 0; q < SEL_REG; q++) {
            const uint32_t idx = tid + q * 256;
            loc[q] = idx < N ? base[idx] : worst_rec();
            if (better(loc[q], v)) v = loc[q];
        }
        const bool has = tid < N;
        const uint32_t rw = wave_rank(v, v, __ballot(has));
        if (has && rw < K) sh.small.wtop[wv][rw] = v;
        if (!has && (uint32_t)lane < K) sh.small.wtop[wv][lane] = worst_rec(); // ranks of real lanes come first
        if (tid == 0) sh.small.ccount = 0;
        __syncthreads();
        const uint32_t nreal = N < 256 ? N : 256; // threads holding at least one record
        const uint32_t Kp = K < nreal ? K : nreal;
        if (tid < 4 * K) {
            const trec me = sh.small.wtop[tid / K][tid % K];
            if (better(me, worst_rec())) {
                uint32_t rank = 0;
                for (uint32_t t = 0; t < 4 * K; t++) rank += better(sh.small.wtop[t / K][t % K], me) ? 1u : 0u;
                if (rank == Kp - 1) sh.small.x = me;
            }
        }
        __syncthreads();
        const trec x = sh.small.x;
#pragma unroll
        for (uint32_t q = 0; q < SEL_REG; q++) {
            if (tid + q * 256 < N && !better(x, loc[q])) {
                const uint32_t slot = atomicAdd(&sh.small.ccount, 1u);
                sh.small.cand[slot] = loc[q];
            }
        }
        __syncthreads();
        const uint32_t C = sh.small.ccount;
        for (uint32_t t = tid; t < C; t += 256) {
            const trec me = sh.small.cand[t];
            uint32_t rank = 0;
            for (uint32_t u = 0; u < C; u++) rank += better(sh.small.cand[u], me) ? 1u : 0u;
            if (rank < K) {
                if (out) put_result(me, off, mode, out + rank);
                if (kth && rank == K - 1) *kth = me;
            }
        }
        __syncthreads();
        return;
    }
    for (uint32_t r0 = 0; r0 < N; r0 += blockDim.x) {
        const uint32_t idx = r0 + tid;
        const bool has = idx < N;
        trec me;
        if (has) me = base[idx];
        uint32_t rank = 0;
        for (uint32_t t0 = 0; t0 < N; t0 += SEL_TILE) {
            const uint32_t cover = N - t0 < SEL_TILE ? N - t0 : SEL_TILE;
            __syncthreads();
            for (uint32_t t = tid; t < cover; t += blockDim.x) sh.tile[t] = base[t0 + t];
            __syncthreads();
            if (has)
                for (uint32_t t = 0; t < cover; t++) rank += better(sh.tile[t], me) ? 1u : 0u;
        }
        if (has && rank < K) {
            if (out) put_result(me, off, mode, out + rank);
            if (kth && rank == K - 1) *kth = me;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ bool wave_selects(uint32_t N, uint32_t K) { return K <= SEL_ROUNDS && N <= WSEL_MAX; }

// Per-graph top-k of the triangles held (graphs with only[g] == 0 skipped when `only` is set),
// one wave per graph: the first min(k, N) triangles with local ids, or n_out[g] = OVERFLOWED
// when the graph's region overflowed.  Graphs with more records than a wave selects from are
// left to k_bselect_big.
__global__ __launch_bounds__(256) void k_bselect(const trec *rec, uint32_t R, const unsigned long long *gcount,
                                                 const uint8_t *only, uint32_t count, uint32_t k, int mode,
                                                 const uint64_t *voff, tt_triangle *out, uint32_t *n_out) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t g = wave; g < count; g += nwaves) {
        if (only && !only[g]) continue;
        const unsigned long long cnt = gcount[g];
        if (cnt > R) {
            if (lane == 0) n_out[g] = OVERFLOWED;
            continue;
        }
        const uint32_t N = (uint32_t)cnt, K = N < k ? N : k;
        if (!wave_selects(N, K)) continue;
        if (K) wave_topk(rec + (uint64_t)g * R, N, K, (uint32_t)voff[g], mode, out + (uint64_t)g * k);
        for (uint32_t r = K + lane; r < k; r += 64) out[(uint64_t)g * k + r] = tt_triangle{0, 0, 0, 0, 0.0};
        if (lane == 0) n_out[g] = K;
    }
}

// The graphs k_bselect leaves: one block per graph.
__global__ __launch_bounds__(256) void k_bselect_big(const trec *rec, uint32_t R, const unsigned long long *gcount,
                                                     const uint8_t *only, uint32_t count, uint32_t k, int mode,
                                                     const uint64_t *voff, tt_triangle *out, uint32_t *n_out) {
    __shared__ SelShared sh;
    for (uint32_t g = blockIdx.x; g < count; g += gridDim.x) {
        if (only && !only[g]) continue;
        const unsigned long long cnt = gcount[g];
        if (cnt > R) continue;
        const uint32_t N = (uint32_t)cnt, K = N < k ? N : k;
        if (wave_selects(N, K)) continue;
        block_topk(rec + (uint64_t)g * R, N, K, (uint32_t)voff[g], mode, out + (uint64_t)g * k, nullptr, sh);
        for (uint32_t r = K + threadIdx.x; r < k; r += blockDim.x) out[(uint64_t)g * k + r] = tt_triangle{0, 0, 0, 0, 0.0};
        if (threadIdx.x == 0) n_out[g] = K;
    }
}

// One restart round, per graph: a graph whose region overflowed (gcount > R) is redone above
// the k-th best full key among the R records it kept (a valid lower bound on its k-th best
// triangle): band [that key, +inf), streaming the segment entries whose bound reaches the
// key's score floor; redo[g] = 1.  Every other graph streams nothing (redo[g] = 0).
__global__ __launch_bounds__(256) void k_brestart(const trec *rec, uint32_t R, unsigned long long *gcount,
                                                  uint32_t count, uint32_t k, int mode, double p,
                                                  const uint64_t *boff, Band *bands, uint32_t *Eg, uint8_t *redo,
                                                  unsigned long long *stats) {
    __shared__ SelShared sh;
    __shared__ trec kth;
    for (uint32_t g = blockIdx.x; g < count; g += gridDim.x) {
        const unsigned long long cnt = gcount[g];
        if (cnt <= R) {
            if (threadIdx.x == 0) {
                Eg[g] = 0;
                redo[g] = 0;
            }
            continue;
        }
        block_topk(rec + (uint64_t)g * R, R, k, 0, mode, nullptr, &kth, sh);
        __syncthreads();
        if (threadIdx.x == 0) {
            Band B;
            B.L = ((u128)kth.khi << 64) | kth.klo;
            B.Li = kth.i;
            B.Lj = kth.j;
            B.Ll = kth.l;
            B.U = 0;
            B.hasU = 0;
            B.mode = mode;
            B.p = p;
            B.theta = mode == MODE_GEN ? key_as_double(B.L) : 0.0;
            bands[g] = B;
            const uint64_t *bo = boff + (uint64_t)g * NB;
            const uint64_t f = score_floor(mode, B.L); // base entries of the band have bound >= f
            Eg[g] = f <= 0xFFFFFFFFull ? (uint32_t)(bo[NB - coarse_bin((uint32_t)f)] - bo[0]) : 0u;
            gcount[g] = 0;
            redo[g] = 1;
            stat_add(stats, 5, 1); // counter 5: graphs restarted
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------- host side
struct BatchCfg {
    uint32_t growth;        // rank ratio between consecutive bands
    uint32_t filter_mul;    // filter blocks per CU
    uint32_t inter_mul;     // intersect blocks per CU
    uint32_t merge_max;     // intersection choice: rows up to this many entries together are merged
};
const BatchCfg CONFIGS[] = {
    {4, 4, 4, 0},    {4, 4, 8, 0},    {4, 16, 4, 0},    {4, 16, 8, 0},    {16, 4, 4, 0},    {16, 4, 8, 0},
    {4, 4, 4, 64},   {4, 4, 8, 64},   {4, 16, 4, 64},   {4, 16, 8, 64},   {16, 4, 4, 64},   {16, 4, 8, 64},
    {4, 4, 4, 256},  {4, 4, 8, 256},  {16, 4, 4, 256},  {16, 4, 8, 256},
};
constexpr int NCONFIGS = (int)(sizeof(CONFIGS) / sizeof(CONFIGS[0]));
constexpr uint32_t IN_GRAPH_RESTARTS = 2; // default restart rounds inside the captured sequence

// A launch choice: configuration, number of passes (the last one exhaustive) and restart
// rounds captured after the selection.
struct Choice {
    int ci;
    uint32_t passes, rounds;
};

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
    // bound-ordered segments for the two most recent p
    struct Order {
        bool valid = false;
        uint64_t pb = 0, last_use = 0;
        uint64_t *boff = nullptr; // [count*NB+1] exclusive prefix of bucket sizes
        uint64_t *goff = nullptr; // [count+1] start of graph g's segment (= boff[g*NB])
        uint32_t *src = nullptr, *col = nullptr, *wgt = nullptr;
    } ord[2];
    uint64_t clock = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    // query state (sized for the largest k seen)
    uint32_t R = 0, kcap = 0;
    Band *bands = nullptr;
    BState *st = nullptr;
    uint32_t *Eg = nullptr;
    uint64_t *poff = nullptr;
    unsigned long long *gcount = nullptr;
    trec *rec = nullptr;
    cand *C = nullptr;
    uint32_t *ccnt = nullptr;
    unsigned long long *spart = nullptr, *dstat = nullptr;
    tt_triangle *dout = nullptr;
    uint32_t *dn = nullptr;
    uint8_t *redo = nullptr;
    // pinned host staging of the results (one device-to-host pass per query)
    uint32_t *h_n = nullptr;
    tt_triangle *h_out = nullptr;
    unsigned long long *h_stat = nullptr;
    unsigned long long extra[6] = {}; // counters of the host-driven restart rounds of the latest query
    hipEvent_t ev[2] = {};
    struct Plan {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        uint32_t passes = 0;
    };
    // (k, bits of p, config, passes, restart rounds) -> captured sequence
    std::map<std::tuple<uint32_t, uint64_t, int, uint32_t, uint32_t>, Plan> plans;
    std::map<std::pair<uint32_t, uint64_t>, Choice> tuned; // (k, bits of p) -> autotuned choice
    std::mutex mu;
};

namespace {

uint64_t p_bits(double p) {
    uint64_t b;
    std::memcpy(&b, &p, 8);
    return b;
}

void free_query_state(tt_batch *b) {
    void *ptrs[] = {b->bands, b->st, b->Eg, b->poff, b->gcount, b->rec, b->C, b->ccnt,
                    b->spart, b->dstat, b->dout, b->dn, b->redo};
    for (void *p : ptrs) dev_free(nullptr, p, 0);
    void *pinned[] = {b->h_n, b->h_out, b->h_stat};
    for (void *p : pinned)
        if (p) (void)hipHostFree(p);
    b->h_n = nullptr;
    b->h_out = nullptr;
    b->h_stat = nullptr;
    b->bands = nullptr; b->st = nullptr; b->Eg = nullptr; b->poff = nullptr; b->gcount = nullptr;
    b->rec = nullptr; b->C = nullptr; b->ccnt = nullptr; b->spart = b->dstat = nullptr;
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
        (rc = dev_alloc(nullptr, (void **)&b->C, (m + 1) * sizeof(cand))) ||
        (rc = dev_alloc(nullptr, (void **)&b->ccnt, MAX_SEG * 4)) ||
        (rc = dev_alloc(nullptr, (void **)&b->spart, 6 * STAT_SLOTS * 8)) ||
        (rc = dev_alloc(nullptr, (void **)&b->dstat, 16 * 8)) ||
        (rc = dev_alloc(nullptr, (void **)&b->dout, n * k * sizeof(tt_triangle) + 8)) ||
        (rc = dev_alloc(nullptr, (void **)&b->dn, n * 4)) ||
        (rc = dev_alloc(nullptr, (void **)&b->redo, n + 1))) {
        free_query_state(b);
        return rc;
    }
    if (hipHostMalloc((void **)&b->h_n, (n + 1) * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->h_out, n * k * sizeof(tt_triangle) + 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->h_stat, 16 * 8, hipHostMallocDefault) != hipSuccess) {
        free_query_state(b);
        return fail(TT_E_NOMEM, "hipHostMalloc failed");
    }
    HIP_TRY(hipMemsetAsync(b->spart, 0, 6 * STAT_SLOTS * 8, b->stream));
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

EnumArgs batch_args(const tt_batch *b, const tt_batch::Order &o, double p, const BatchCfg &c) {
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
    A.vi = g->vinfo;
    A.cw = g->cw;
    A.merge_max = c.merge_max;
    A.scan_max = SCAN_MAX;
    A.s_src = o.src;
    A.s_col = o.col;
    A.s_wgt = o.wgt;
    A.B.mode = mode_of(p);
    A.B.p = p;
    A.out = b->rec;
    A.stats = b->spart;
    A.C = b->C;
    A.ccnt = b->ccnt;
    A.nseg = std::min<uint32_t>((uint32_t)num_cus() * c.filter_mul, MAX_SEG);
    A.bands = b->bands;
    A.poff = b->poff;
    A.goff = o.goff;
    A.ng = b->count;
    A.gcount = b->gcount;
    A.R = b->R;
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
    const unsigned igrid = (unsigned)num_cus() * c.inter_mul;
    if (A.B.mode == MODE_GEN) {
        k_filter<FILTER_NONE, true, true><<<A.nseg, 256, 0, s>>>(A);
        k_intersect<FILTER_NONE, true, true><<<igrid, 256, 0, s>>>(A);
    } else {
        k_filter<FILTER_NONE, true, false><<<A.nseg, 256, 0, s>>>(A);
        k_intersect<FILTER_NONE, true, false><<<igrid, 256, 0, s>>>(A);
    }
    HIP_TRY(hipGetLastError());
    return TT_OK;
}

unsigned sel_grid(const tt_batch *b) { return std::min<unsigned>(b->count, (unsigned)num_cus() * 8); }

// Per-graph selection: a wave per graph, then a block per graph for the few with many records.
void enqueue_select(tt_batch *b, uint32_t k, int mode, const uint8_t *only) {
    hipStream_t s = b->stream;
    k_bselect<<<(b->count + 3) / 4, 256, 0, s>>>(b->rec, b->R, b->gcount, only, b->count, k, mode, b->voff, b->dout,
                                                  b->dn);
    k_bselect_big<<<sel_grid(b), 256, 0, s>>>(b->rec, b->R, b->gcount, only, b->count, k, mode, b->voff, b->dout,
                                              b->dn);
}

int enqueue_restart_round(tt_batch *b, const EnumArgs &A, const BatchCfg &c, uint32_t k, double p,
                          const tt_batch::Order &o) {
    hipStream_t s = b->stream;
    const int mode = mode_of(p);
    k_brestart<<<sel_grid(b), 256, 0, s>>>(b->rec, b->R, b->gcount, b->count, k, mode, p, o.boff, b->bands, b->Eg,
                                           b->redo, b->spart);
    int rc = enqueue_pass(b, A, c);
    if (rc) return rc;
    enqueue_select(b, k, mode, b->redo);
    HIP_TRY(hipGetLastError());
    return TT_OK;
}

// The launch sequence of one query: every pass of the descent, then the per-graph selection
// and the counters.  Nothing in it allocates, copies or sets memory, so it can be captured.
int enqueue_query(tt_batch *b, const tt_batch::Order &o, uint32_t k, double p, const BatchCfg &c, uint32_t P,
                  uint32_t rounds) {
    hipStream_t s = b->stream;
    const int mode = mode_of(p);
    EnumArgs A = batch_args(b, o, p, c);
    const unsigned pg = (b->count + 255) / 256;
    unsigned long long M = k;
    for (uint32_t i = 0; i < P; i++) {
        const unsigned long long Mi = i + 1 == P ? ~0ull : M; // the last band is exhaustive
        k_bplan<<<pg, 256, 0, s>>>(i, b->count, k, mode, p, Mi, o.boff, b->gcount, b->st, b->bands, b->Eg);
        int rc = enqueue_pass(b, A, c);
        if (rc) return rc;
        M = M > (~0ull / c.growth) ? ~0ull : M * c.growth;
    }
    enqueue_select(b, k, mode, nullptr);
    // restart rounds decided on the device: graphs whose region overflowed are redone above the
    // k-th best key they hold; a round with nothing to redo streams nothing
    for (uint32_t round = 0; round < rounds; round++) {
        int rc = enqueue_restart_round(b, A, c, k, p, o);
        if (rc) return rc;
    }
    k_reduce_stats<<<6, 256, 0, s>>>(b->spart, b->dstat);
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
            (rc = dev_alloc(nullptr, (void **)&b->gm, (count + 1) * 8)))
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

// The bound-ordered segments for p (built on first use, the two most recent p kept).  Plans
// captured for the p whose segments are replaced are dropped with them.
int ensure_order(tt_batch *b, double p, const tt_batch::Order **out) {
    const uint64_t pb = p_bits(p);
    b->clock++;
    for (auto &o : b->ord)
        if (o.valid && o.pb == pb) {
            o.last_use = b->clock;
            *out = &o;
            return TT_OK;
        }
    tt_batch::Order &o = b->ord[0].last_use <= b->ord[1].last_use ? b->ord[0] : b->ord[1];
    if (o.valid) {
        for (auto it = b->plans.begin(); it != b->plans.end();) {
            if (std::get<1>(it->first) == o.pb) {
                (void)hipGraphExecDestroy(it->second.exec);
                (void)hipGraphDestroy(it->second.graph);
                it = b->plans.erase(it);
            } else {
                ++it;
            }
        }
    }
    o.valid = false;
    const uint64_t count = b->count, M = b->g->m, nb = count * NB + 1;
    int rc;
    if (!o.src && ((rc = dev_alloc(nullptr, (void **)&o.boff, nb * 8)) ||
                   (rc = dev_alloc(nullptr, (void **)&o.goff, (count + 1) * 8)) ||
                   (rc = dev_alloc(nullptr, (void **)&o.src, (M + 1) * 4)) ||
                   (rc = dev_alloc(nullptr, (void **)&o.col, (M + 1) * 4)) ||
                   (rc = dev_alloc(nullptr, (void **)&o.wgt, (M + 1) * 4))))
        return rc;
    hipStream_t s = b->stream;
    uint32_t *bcnt = nullptr;
    if ((rc = dev_alloc(nullptr, (void **)&bcnt, nb * 4))) return rc;
    const tt_graph *g = b->g;
    const int mode = mode_of(p);
    auto body = [&]() -> int {
        HIP_TRY(hipMemsetAsync(bcnt, 0, nb * 4, s));
        HIP_TRY(hipMemsetAsync(o.goff, 0, (count + 1) * 8, s));
        k_ocount<<<(unsigned)count, 256, 0, s>>>(b->voff, g->rstart, g->rlen, g->col, g->wgt, g->maxw, mode, p, bcnt);
        HIP_TRY(hipGetLastError());
        int r2 = exclusive_scan_u32_to_u64(bcnt, o.boff, nb, s, nullptr);
        if (r2) return r2;
        k_oscatter<<<(unsigned)count, 256, 0, s>>>(b->voff, g->rstart, g->rlen, g->col, g->wgt, g->maxw, mode, p,
                                                  o.boff, o.src, o.col, o.wgt);
        k_goff<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(o.boff, (uint32_t)count, o.goff);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        return TT_OK;
    };
    rc = body();
    (void)hipStreamSynchronize(s);
    dev_free(nullptr, bcnt, 0);
    if (rc) return rc;
    o.valid = true;
    o.pb = pb;
    o.last_use = b->clock;
    *out = &o;
    return TT_OK;
}

// Runs one query with configuration c: replays (or first captures) its plan, or enqueues it
// directly when `eager`; then redoes overflowed graphs.  Results stay in b->dout / b->dn.
int run_batch(tt_batch *b, uint32_t k, double p, const Choice &ch, bool eager, double *ms) {
    const BatchCfg &c = CONFIGS[ch.ci];
    hipStream_t s = b->stream;
    const tt_batch::Order *o = nullptr;
    int rc;
    if ((rc = ensure_order(b, p, &o))) return rc;
    HIP_TRY(hipEventRecord(b->ev[0], s));
    if (eager) {
        if ((rc = enqueue_query(b, *o, k, p, c, ch.passes, ch.rounds))) return rc;
    } else {
        auto key = std::make_tuple(k, p_bits(p), ch.ci, ch.passes, ch.rounds);
        auto it = b->plans.find(key);
        if (it == b->plans.end()) {
            tt_batch::Plan pl;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            rc = enqueue_query(b, *o, k, p, c, ch.passes, ch.rounds);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (e != hipSuccess) return fail(TT_E_DEVICE, std::string("stream capture: ") + hipGetErrorString(e));
            pl.graph = graph;
            HIP_TRY(hipGraphInstantiate(&pl.exec, graph, nullptr, nullptr, 0));
            pl.passes = ch.passes;
            it = b->plans.emplace(key, pl).first;
        }
        HIP_TRY(hipGraphLaunch(it->second.exec, s));
    }
    HIP_TRY(hipEventRecord(b->ev[1], s));
    std::memset(b->extra, 0, sizeof(b->extra));
    const uint64_t out_bytes = (uint64_t)b->count * k * sizeof(tt_triangle);
    auto fetch = [&](const unsigned long long *dstat, unsigned long long *hstat) -> int {
        HIP_TRY(hipMemcpyAsync(b->h_n, b->dn, (uint64_t)b->count * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(b->h_out, b->dout, out_bytes, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hstat, dstat, 6 * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return TT_OK;
    };
    if ((rc = fetch(b->dstat, b->h_stat))) return rc;
    if (ms) {
        float f = 0.f;
        (void)hipEventElapsedTime(&f, b->ev[0], b->ev[1]);
        *ms = f;
    }
    // graphs whose region overflowed: redo above the k-th best key they hold
    EnumArgs A = batch_args(b, *o, p, c);
    for (int round = 0; round < 64; round++) {
        bool any = false;
        for (uint32_t g = 0; g < b->count && !any; g++) any = b->h_n[g] == OVERFLOWED;
        if (!any) return TT_OK;
        if ((rc = enqueue_restart_round(b, A, c, k, p, *o))) return rc;
        k_reduce_stats<<<6, 256, 0, s>>>(b->spart, b->dstat + 8);
        HIP_TRY(hipGetLastError());
        if ((rc = fetch(b->dstat + 8, b->h_stat + 8))) return rc;
        for (int c2 = 0; c2 < 6; c2++) b->extra[c2] += b->h_stat[8 + c2];
    }
    return fail(TT_E_DEVICE, "batched query: overflow restarts did not converge");
}

// Mean device time of a few replays of choice ch (after one capture / warm-up run).
int time_choice(tt_batch *b, uint32_t k, double p, const Choice &ch, double *out) {
    double ms = 0, tot = 0;
    int rc = run_batch(b, k, p, ch, false, &ms);
    if (rc) return rc;
    for (int r = 0; r < 3; r++) {
        if ((rc = run_batch(b, k, p, ch, false, &ms))) return rc;
        tot += ms;
    }
    *out = tot / 3;
    return TT_OK;
}

// Picks, by timing replays: the launch configuration (all passes, default restart rounds),
// then the number of passes (fewer passes make the exhaustive last one larger), then the
// number of restart rounds captured (rounds not captured run from the host when needed).
// Every choice returns the same result.
int autotune(tt_batch *b, uint32_t k, double p, Choice *best, double *tune_ms) {
    const double t0 = now_ms();
    double best_ms = 1e300, ms = 0;
    Choice bc{0, 0, IN_GRAPH_RESTARTS};
    int rc;
    for (int ci = 0; ci < NCONFIGS; ci++) {
        const Choice ch{ci, passes_for(b, k, CONFIGS[ci].growth), IN_GRAPH_RESTARTS};
        if ((rc = time_choice(b, k, p, ch, &ms))) return rc;
        if (ms < best_ms) { best_ms = ms; bc = ch; }
    }
    int worse = 0;
    for (uint32_t P = bc.passes; P-- > 1 && worse < 2;) {
        const Choice ch{bc.ci, P, bc.rounds};
        if ((rc = time_choice(b, k, p, ch, &ms))) return rc;
        if (ms < best_ms) { best_ms = ms; bc = ch; worse = 0; } else worse++;
    }
    for (uint32_t r = 0; r < IN_GRAPH_RESTARTS; r++) {
        const Choice ch{bc.ci, bc.passes, r};
        if ((rc = time_choice(b, k, p, ch, &ms))) return rc;
        if (ms < best_ms) { best_ms = ms; bc = ch; }
    }
    // plans that lost are released
    for (auto it = b->plans.begin(); it != b->plans.end();) {
        const auto &key = it->first;
        if (std::get<0>(key) == k && std::get<1>(key) == p_bits(p) &&
            !(std::get<2>(key) == bc.ci && std::get<3>(key) == bc.passes && std::get<4>(key) == bc.rounds)) {
            (void)hipGraphExecDestroy(it->second.exec);
            (void)hipGraphDestroy(it->second.graph);
            it = b->plans.erase(it);
        } else {
            ++it;
        }
    }
    *best = bc;
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
    if (k == 0 || b->count == 0 || b->g->m == 0) {
        if (k && out) std::memset(out, 0, (uint64_t)b->count * k * sizeof(tt_triangle));
        set_error("");
        return TT_OK;
    }
    std::lock_guard<std::mutex> lock(b->mu);
    (void)hipSetDevice(b->g->device);
    int rc = ensure_query_state(b, k);
    if (rc) return rc;
    Choice ch{config, 0, IN_GRAPH_RESTARTS};
    double tune_ms = 0.0;
    if (config < 0) {
        auto key = std::make_pair(k, p_bits(p));
        auto it = b->tuned.find(key);
        if (it == b->tuned.end()) {
            if ((rc = autotune(b, k, p, &ch, &tune_ms))) return rc;
            b->tuned[key] = ch;
        } else {
            ch = it->second;
        }
    } else {
        ch.passes = passes_for(b, k, CONFIGS[config].growth);
    }
    const int ci = ch.ci;
    double ms = 0.0;
    if ((rc = run_batch(b, k, p, ch, (flags & TT_BATCH_EAGER) != 0, &ms))) return rc;
    std::memcpy(n_out, b->h_n, (uint64_t)b->count * 4);
    std::memcpy(out, b->h_out, (uint64_t)b->count * k * sizeof(tt_triangle));
    const unsigned long long *st = b->h_stat;
    if (stats) {
        stats->config = (uint32_t)ci;
        stats->growth = CONFIGS[ci].growth;
        stats->filter_blocks = std::min<uint32_t>((uint32_t)num_cus() * CONFIGS[ci].filter_mul, MAX_SEG);
        stats->intersect_blocks = (uint32_t)num_cus() * CONFIGS[ci].inter_mul;
        stats->passes = ch.passes;
        stats->restart_rounds = ch.rounds;
        stats->merge_max = CONFIGS[ci].merge_max;
        stats->restarts = (uint32_t)(st[5] + b->extra[5]);
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
    for (auto &o : b->ord) {
        void *op[] = {o.boff, o.goff, o.src, o.col, o.wgt};
        for (void *p : op) dev_free(nullptr, p, 0);
    }
    void *ptrs[] = {b->voff, b->gm};
    for (void *p : ptrs) dev_free(nullptr, p, 0);
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->g) graph_free(b->g);
    if (b->owns_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}
