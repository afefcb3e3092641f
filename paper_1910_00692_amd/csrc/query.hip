// query.hip — exact top-k triangles (Sec. 1 problem, Eq. 1 scores) and weighted edge
// sampling (Alg. 3) on a loaded graph.
//
// Pruned enumeration.  Sec. 3.2 bounds the heaviest triangle that has not been enumerated
// from the weights of the edges not yet processed.  The same monotonicity gives, for any
// threshold L on the order key: a triangle (u,v,c) reached at oriented entry u->v has weights
// a = w_uv, x = w_uc <= maxw(u), y = w_vc <= maxw(v), so it can reach L only if
// key(a, maxw(u), maxw(v)) >= L (entry filter), and then only entries with
// x >= min{x : key(a, x, maxw(v)) >= L} (and symmetrically for y) can take part.  m_p is
// non-decreasing in each argument for every p in [-inf, +inf], so this holds for all p.
//
// Threshold descent.  Instead of the sequential pointer walk of Alg. 2, the host runs a short
// sequence of data-parallel passes over decreasing score bands [L_i, L_{i-1}), with L_i taken
// from quantiles of the edge-weight distribution (the k-th, 4k-th, 16k-th ... heaviest edge,
// as in the heavy/light split of Sec. 3).  Bands are disjoint, so after pass i the candidate
// buffer holds exactly the triangles with key >= L_i; as soon as it holds >= k of them the
// top-k is among them (the argument of Sec. 3.2).  If the buffer overflows, its k-th best full
// key (score, i, j, l) is a valid lower bound and the pass is redone above it.
//
// Selection.  The buffer is sorted in LDS tiles of 1024 records by (key desc, i, j, l asc),
// each tile truncated to k, then merged pairwise (every record finds its rank in the sibling
// run by binary search) with runs truncated to k, down to one run.
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <new>
#include <thread>
#include <unordered_map>

#include "common.h"
#include "enum.h"
#include "scan.h"
#include "serve_core.h"

namespace {

// ----------------------------------------------------------------------------- selection
constexpr int STILE = 1024;


// Sorts each tile of STILE records (best first) and keeps its first S0.  Thread t holds the
// records at positions t and t + 512 in registers; a bitonic compare-exchange at stride s pairs
// positions i and i ^ s: below 64 the partner is in the same wave (shuffles of the record's
// seven words), from 64 to 256 in another wave (an exchange through LDS), at 512 in the same
// thread.
__device__ __forceinline__ trec shfl_xor_rec(const trec &r, int s) {
    trec o;
    o.khi = ((uint64_t)__shfl_xor((uint32_t)(r.khi >> 32), s, 64) << 32) | __shfl_xor((uint32_t)r.khi, s, 64);
    o.klo = ((uint64_t)__shfl_xor((uint32_t)(r.klo >> 32), s, 64) << 32) | __shfl_xor((uint32_t)r.klo, s, 64);
    o.i = __shfl_xor(r.i, s, 64);
    o.j = __shfl_xor(r.j, s, 64);
    o.l = __shfl_xor(r.l, s, 64);
    o.pad = 0;
    return o;
}

__global__ __launch_bounds__(512) void k_tile_sort(const trec *in, trec *out, uint64_t N, uint32_t S0) {
    static_assert(STILE == 1024, "two records per thread of a 512-thread block");
    __shared__ trec xch[STILE];
    const uint32_t t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x * STILE;
    const uint32_t cover = (uint32_t)((N - base) < (uint64_t)STILE ? (N - base) : (uint64_t)STILE);
    trec r[2];
    r[0] = t < cover ? in[base + t] : worst_rec();
    r[1] = t + 512 < cover ? in[base + t + 512] : worst_rec();
#pragma unroll
    for (uint32_t size = 2; size <= (uint32_t)STILE; size <<= 1) {
#pragma unroll
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride == 512) { // size 1024: the better record goes first everywhere
                if (better(r[1], r[0])) { const trec x = r[0]; r[0] = r[1]; r[1] = x; }
                continue;
            }
            trec o[2];
            if (stride >= 64) {
                __syncthreads();
                xch[t] = r[0];
                xch[t + 512] = r[1];
                __syncthreads();
                o[0] = xch[t ^ stride];
                o[1] = xch[(t + 512) ^ stride];
            } else {
                o[0] = shfl_xor_rec(r[0], (int)stride);
                o[1] = shfl_xor_rec(r[1], (int)stride);
            }
#pragma unroll
            for (int q = 0; q < 2; q++) {
                const uint32_t i = t + 512u * q;
                // the lower position of a pair takes the better record where (i & size) == 0
                const bool keep_better = ((i & stride) == 0) == ((i & size) == 0);
                if (better(o[q], r[q]) == keep_better) r[q] = o[q];
            }
        }
    }
    const uint32_t keep = cover < S0 ? cover : S0;
    if (t < keep) out[(uint64_t)blockIdx.x * S0 + t] = r[0];
    if (t + 512 < keep) out[(uint64_t)blockIdx.x * S0 + t + 512] = r[1];
}

// Merges runs 2r and 2r+1 (cover C, stride S) into run r (stride So), keeping the first So.
__global__ __launch_bounds__(256) void k_merge(const trec *in, trec *out, uint64_t N, uint64_t C, uint32_t S,
                                               uint32_t So, uint64_t nruns) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t rp = gid / (2ull * S);
    const uint32_t x = (uint32_t)(gid % (2ull * S));
    const uint64_t ra = 2 * rp, rb = ra + 1;
    if (ra >= nruns) return;
    const uint64_t cova = (N - ra * C) < C ? (N - ra * C) : C;
    const uint32_t La = (uint32_t)(cova < S ? cova : S);
    uint32_t Lb = 0;
    if (rb < nruns) {
        const uint64_t covb = (N - rb * C) < C ? (N - rb * C) : C;
        Lb = (uint32_t)(covb < S ? covb : S);
    }
    const bool isA = x < S;
    const uint32_t idx = isA ? x : x - S;
    if (idx >= (isA ? La : Lb)) return;
    const trec me = in[(isA ? ra : rb) * S + idx];
    const trec *sib = in + (isA ? rb : ra) * S;
    uint32_t lo = 0, hi = isA ? Lb : La;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (better(sib[mid], me)) lo = mid + 1; else hi = mid;
    }
    const uint64_t pos = (uint64_t)idx + lo;
    if (pos < So) out[rp * So + pos] = me;
}

__global__ void k_finalize(const trec *in, uint32_t K, int mode, tt_triangle *out) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K) return;
    const trec r = in[t];
    tt_triangle o;
    o.i = r.i; o.j = r.j; o.l = r.l; o._pad = 0;
    o.score = key_to_score(mode, ((u128)r.khi << 64) | r.klo);
    out[t] = o;
}

// ----------------------------------------------------------------------------- sampling
// s-th output (0-based) of SplitMix64 started from state `seed` (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t s) {
    uint64_t z = seed + (s + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The draw rule: the edge picked by the 64-bit uniform x is the first e with prefix[e] > r(x),
// r(x) = floor(x * Z / 2^64) (integer prefix) or (x >> 11) * 2^-53 * Z (FP64 prefix).
// KIND 0: u64 prefix (q = 1); 1: u128 prefix (q = 2, 3); 2: FP64 prefix.
template <int KIND> struct Draw;
template <> struct Draw<0> {
    typedef uint64_t T;
    static __device__ __forceinline__ T r(const T *P, uint64_t m, uint64_t x) { return __umul64hi(x, P[m - 1]); }
};
template <> struct Draw<1> {
    typedef u128 T;
    static __device__ __forceinline__ T r(const T *P, uint64_t m, uint64_t x) {
        const u128 Z = P[m - 1];
        return ((u128)x * (uint64_t)(Z >> 64)) + (u128)__umul64hi(x, (uint64_t)Z);
    }
};
template <> struct Draw<2> {
    typedef double T;
    static __device__ __forceinline__ T r(const T *P, uint64_t m, uint64_t x) {
        return (double)(x >> 11) * (1.0 / 9007199254740992.0) * P[m - 1];
    }
};

// first e in [lo, hi] with P[e] > r (the answer is known to lie in that range)
template <typename T> __device__ __forceinline__ uint64_t first_above(const T *P, uint64_t lo, uint64_t hi, T r) {
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (P[mid] > r) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Guide table (cut points): G[j] = the edge picked by x = j * 2^(64-bits), j = 0 .. 2^bits - 1,
// and G[2^bits] = m - 1.  The draw rule is monotone in x, so every x in bucket j picks an edge
// in [G[j], G[j+1]]; a draw then searches only that range, with the same result.
// Each thread fills GUIDE_RUN consecutive cut points: a full search for the first, then a
// galloping search that starts at the previous cut point (the cut points never decrease).
constexpr uint32_t GUIDE_RUN = 4; // measured best among 1, 2, 4, 8 and 16 on the 1M-vertex graph

template <int KIND>
__global__ __launch_bounds__(256) void k_es_guide(const void *prefix, uint64_t m, uint32_t bits, uint32_t *G) {
    typedef typename Draw<KIND>::T T;
    const T *P = (const T *)prefix;
    const uint64_t nb = 1ull << bits, runs = (nb + GUIDE_RUN - 1) / GUIDE_RUN;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= runs; t += (uint64_t)gridDim.x * blockDim.x) {
        if (t == runs) { G[nb] = (uint32_t)(m - 1); continue; }
        const uint64_t j0 = t * GUIDE_RUN, j1 = j0 + GUIDE_RUN < nb ? j0 + GUIDE_RUN : nb;
        uint64_t e = first_above<T>(P, 0, m - 1, Draw<KIND>::r(P, m, j0 << (64 - bits)));
        G[j0] = (uint32_t)e;
        for (uint64_t j = j0 + 1; j < j1; j++) {
            const T r = Draw<KIND>::r(P, m, j << (64 - bits));
            if (e < m - 1 && !(P[e] > r)) {
                // P[lo] <= r; double the step until P[hi] > r or hi reaches m - 1
                uint64_t lo = e, hi, step = 1;
                for (;;) {
                    hi = lo + step;
                    if (hi >= m - 1) { hi = m - 1; break; }
                    if (P[hi] > r) break;
                    lo = hi;
                    step <<= 1;
                }
                e = first_above<T>(P, lo + 1, hi, r);
            }
            G[j] = (uint32_t)e;
        }
    }
}

// Draw s marks the entry of its edge; with `dump` it also records the edge's input index.
template <int KIND>
__global__ __launch_bounds__(256) void k_es_draw(const void *prefix, const uint32_t *G, uint32_t bits, uint64_t m,
                                                 uint64_t budget, uint64_t seed, const uint32_t *opos, uint8_t *emark,
                                                 uint32_t *dump) {
    typedef typename Draw<KIND>::T T;
    const T *P = (const T *)prefix;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < budget; s += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = splitmix64_at(seed, s);
        const uint64_t j = x >> (64 - bits);
        const uint64_t e = first_above<T>(P, G[j], G[j + 1], Draw<KIND>::r(P, m, x));
        emark[opos[e]] = 1;
        if (dump) dump[s] = (uint32_t)e;
    }
}

// vflag[u] = 1 for every tail u with a drawn out-entry (a streaming pass over the marks).
// Also adds the number of drawn entries (distinct sampled edges) to *count: one atomic per block.
__global__ __launch_bounds__(256) void k_mark_tails(const uint8_t *emark, uint64_t m, const uint32_t *osrc,
                                                    uint8_t *vflag, unsigned long long *count) {
    __shared__ unsigned long long part[4];
    const uint64_t nv = (m + 15) / 16;
    unsigned long long c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 x = ((const uint4 *)emark)[i];
        if ((x.x | x.y | x.z | x.w) == 0) continue;
        const uint32_t w[4] = {x.x, x.y, x.z, x.w};
        for (int k = 0; k < 16; k++) {
            const uint64_t e = i * 16 + k;
            if (e < m && ((w[k >> 2] >> ((k & 3) * 8)) & 0xFFu)) {
                vflag[osrc[e]] = 1;
                c++;
            }
        }
    }
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(count, t);
    }
}

// Sets vertex x in a byte-flag array through its 32-bit word; true for the one thread that
// set it first (the arrays are padded to a multiple of four bytes).
__device__ __forceinline__ bool flag_first(uint8_t *flags, uint32_t x) {
    const uint32_t bit = 1u << (8 * (x & 3u));
    const uint32_t old = atomicOr(reinterpret_cast<uint32_t *>(flags + (x & ~3u)), bit);
    return !(old & bit);
}

// Subset queries.  A triangle u->v, u->c, v->c (base u->v) touches the subset S iff u in S, or
// v in S, or c in S; in the last case u and v both have an out-neighbour in S.  So its base is
// (A) an out-entry of a vertex of S, or (B/C) an out-entry u->v of an in-neighbour u of S
// (u outside S) whose head v is in S or has an out-neighbour in S.  The three kernels below mark
// S (vflag), mark every vertex with an out-neighbour in S (vflag2) through the in-rows of S,
// list the in-neighbours outside S, and copy the base entries of those rows into a compact
// stream.  Sources are disjoint, so no entry appears twice.
//
// Marks S and drops repeated ids: own[t] = 1 for the first copy of ids[t]; lens[t] = in-degree
// of an owned id (else 0), lens[cnt] = 0; cnt8[1] += out-degrees of the owned ids.
__global__ __launch_bounds__(256) void k_sub_mark(const uint32_t *ids, uint32_t cnt, const uint64_t *irstart,
                                                  const uint32_t *rlen, uint8_t *vflag, uint8_t *own, uint32_t *lens,
                                                  unsigned long long *cnt8) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long out_sum = 0;
    if (t < cnt) {
        const uint32_t x = ids[t];
        const bool first = flag_first(vflag, x);
        own[t] = first ? 1 : 0;
        lens[t] = first ? (uint32_t)(irstart[x + 1] - irstart[x]) : 0u;
        if (first) out_sum = rlen[x];
    } else if (t == cnt) {
        lens[t] = 0;
    }
    out_sum = wave_sum(out_sum);
    if ((threadIdx.x & 63) == 0 && out_sum) atomicAdd(&cnt8[1], out_sum);
}

// One thread per in-entry u->s of the (owned) subset vertices, flattened through the exclusive
// prefix pre[] of lens[]: sets vflag2[u]; the first setter with u outside S appends u to vlist
// (cnt8[0]) and adds its out-degree to cnt8[1].
__global__ __launch_bounds__(256) void k_sub_in(const uint32_t *ids, uint32_t cnt, const uint64_t *pre,
                                                const uint64_t *irstart, const uint32_t *itail, const uint32_t *rlen,
                                                const uint8_t *vflag, uint8_t *vflag2, uint32_t *vlist, uint64_t vcap,
                                                unsigned long long *cnt8) {
    const int lane = threadIdx.x & 63;
    const uint64_t total = pre[cnt];
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t base = wave * 64; base < total; base += nwaves * 64) {
        const uint64_t idx = base + lane;
        bool app = false;
        uint32_t u = 0;
        if (idx < total) {
            uint32_t lo = 0, hi = cnt; // last t with pre[t] <= idx
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (pre[mid] <= idx) lo = mid; else hi = mid;
            }
            u = itail[irstart[ids[lo]] + (idx - pre[lo])];
            app = flag_first(vflag2, u) && !vflag[u];
        }
        const uint64_t bal = __ballot(app);
        if (bal) {
            unsigned long long b0 = 0;
            if (lane == 0) b0 = atomicAdd(&cnt8[0], (unsigned long long)__popcll(bal));
            b0 = __shfl(b0, 0, 64);
            const uint64_t slot = b0 + __popcll(bal & ((1ull << lane) - 1ull));
            if (app && slot < vcap) vlist[slot] = u;
            const unsigned long long d = wave_sum((unsigned long long)(app ? rlen[u] : 0u));
            if (lane == 0 && d) atomicAdd(&cnt8[1], d);
        }
    }
}

// One wave per row: rows 0..cnt-1 are the subset ids (owned copies only, every entry kept),
// rows cnt..cnt+nv-1 the listed in-neighbours (entries whose head is in S or has an
// out-neighbour in S).  Kept entries go to the compact stream (cnt8[2]) with their weight
// histogram (hist, by weight_bin); the stream's position field holds, for an entry of a listed
// in-neighbour u, u's index in vlist (~0 for a subset row).  A listed row's entries whose head is
// in S are also written, in row order, to one run of sp_c / sp_w reserved for the row (cnt8[3]),
// recorded in sp_start / sp_cnt: the candidate u->v whose triangles must close on a subset
// vertex then looks up only those heads in v's row.
__global__ __launch_bounds__(256) void k_sub_rows(const uint32_t *ids, const uint8_t *own, uint32_t cnt,
                                                  const uint32_t *vlist, uint32_t nv, const uint64_t *rstart,
                                                  const uint32_t *rlen, const uint32_t *col, const uint32_t *wgt,
                                                  const uint8_t *vflag, const uint8_t *vflag2, uint32_t *o_src,
                                                  uint32_t *o_col, uint32_t *o_wgt, uint32_t *o_pos, uint64_t cap,
                                                  uint32_t *sp_c, uint32_t *sp_w, uint32_t *sp_start,
                                                  uint32_t *sp_cnt, unsigned long long *cnt8,
                                                  unsigned long long *hist) {
    __shared__ uint32_t h[WBINS];
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x) h[t] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint64_t rows = (uint64_t)cnt + nv;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < rows; r += nwaves) {
        const bool in_s = r < cnt;
        if (in_s && !own[r]) continue;
        const uint32_t u = in_s ? ids[r] : vlist[r - cnt];
        const uint64_t b = rstart[u];
        const uint32_t len = rlen[u];
        const uint32_t li = in_s ? ~0u : (uint32_t)(r - cnt); // index in vlist
        // a listed row: its heads in S counted first, then one run reserved for them
        uint64_t sp0 = 0;
        uint32_t spn = 0;
        if (!in_s) {
            for (uint32_t t0 = 0; t0 < len; t0 += 64) {
                const uint32_t t = t0 + lane;
                spn += (uint32_t)__popcll(__ballot(t < len && vflag[col[b + t]]));
            }
            unsigned long long s0 = 0;
            if (lane == 0 && spn) s0 = atomicAdd(&cnt8[3], (unsigned long long)spn);
            sp0 = __shfl(s0, 0, 64);
            if (lane == 0) {
                // a run past the capacity is recorded empty (then the kept stream overflows too)
                const bool fits = sp0 + spn <= cap;
                sp_start[li] = fits ? (uint32_t)sp0 : 0u;
                sp_cnt[li] = fits ? spn : 0u;
            }
        }
        uint32_t spr = 0; // heads in S written so far
        for (uint32_t t0 = 0; t0 < len; t0 += 64) {
            const uint32_t t = t0 + lane;
            bool keep = false, ins = false;
            uint32_t v = 0, w = 0;
            if (t < len) {
                v = col[b + t];
                ins = vflag[v];
                keep = in_s || ins || vflag2[v];
                if (keep) w = wgt[b + t];
            }
            if (!in_s) {
                const uint64_t sb = __ballot(ins);
                const uint64_t ps = sp0 + spr + __popcll(sb & ((1ull << lane) - 1ull));
                if (ins && sp0 + spn <= cap) {
                    sp_c[ps] = v;
                    sp_w[ps] = w;
                }
                spr += (uint32_t)__popcll(sb);
            }
            const uint64_t bal = __ballot(keep);
            if (!bal) continue;
            unsigned long long b0 = 0;
            if (lane == 0) b0 = atomicAdd(&cnt8[2], (unsigned long long)__popcll(bal));
            b0 = __shfl(b0, 0, 64);
            const uint64_t slot = b0 + __popcll(bal & ((1ull << lane) - 1ull));
            if (keep && slot < cap) {
                o_src[slot] = u;
                o_col[slot] = v;
                o_wgt[slot] = w;
                o_pos[slot] = li;
                atomicAdd(&h[weight_bin(w)], 1u);
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x)
        if (h[t]) atomicAdd(&hist[t], (unsigned long long)h[t]);
}

// ----------------------------------------------------------------------------- bound order

// Entries per bin of their bound (an integer >= m_p(w_uv, maxw(u), maxw(v))).
__global__ __launch_bounds__(256) void k_bound_hist(const uint32_t *osrc, const uint32_t *col, const uint32_t *wgt,
                                                    const uint32_t *maxw, uint64_t m, int mode, double p,
                                                    unsigned long long *hist) {
    __shared__ uint32_t h[WBINS];
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x) h[t] = 0;
    __syncthreads();
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[weight_bin(entry_bound(mode, p, wgt[e], maxw[osrc[e]], maxw[col[e]]))], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x)
        if (h[t]) atomicAdd(&hist[t], (unsigned long long)h[t]);
}

// Entries grouped by descending bound bin.  A block places a chunk of BPLACE_CHUNK consecutive
// entries: their bins are kept in LDS, one global atomic per (block, non-empty bin) reserves
// the block's run inside each bin, and an LDS cursor per bin hands out slots, so the entries
// of one bin from one block land in one contiguous run (whole cache lines, not scattered words).
constexpr uint32_t BPLACE_CHUNK = 16384;
__global__ __launch_bounds__(256) void k_place_bound(const uint32_t *osrc, const uint32_t *col, const uint32_t *wgt,
                                                     const uint32_t *maxw, uint64_t m, int mode, double p,
                                                     const unsigned long long *binbase, unsigned long long *bincur,
                                                     uint32_t *o_src, uint32_t *o_col, uint32_t *o_wgt,
                                                     uint32_t *o_pos) {
    __shared__ uint16_t bins[BPLACE_CHUNK];
    __shared__ uint32_t lc[WBINS];
    __shared__ unsigned long long lb[WBINS];
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x) lc[t] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * BPLACE_CHUNK;
    const uint32_t cover = (uint32_t)(m - base < BPLACE_CHUNK ? m - base : BPLACE_CHUNK);
    for (uint32_t t = threadIdx.x; t < cover; t += blockDim.x) {
        const uint64_t e = base + t;
        const uint32_t b = weight_bin(entry_bound(mode, p, wgt[e], maxw[osrc[e]], maxw[col[e]]));
        bins[t] = (uint16_t)b;
        atomicAdd(&lc[b], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x) {
        if (lc[t]) lb[t] = binbase[t] + atomicAdd(&bincur[t], (unsigned long long)lc[t]);
        lc[t] = 0;
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < cover; t += blockDim.x) {
        const uint64_t e = base + t;
        const uint32_t b = bins[t];
        const uint64_t d = lb[b] + atomicAdd(&lc[b], 1u);
        o_src[d] = osrc[e];
        o_col[d] = col[e];
        o_wgt[d] = wgt[e];
        o_pos[d] = (uint32_t)e;
    }
}

// ----------------------------------------------------------------------------- host side
// Candidates whose two rows hold at most this many entries together are intersected by a
// lane-local merge (sequential reads of both rows) instead of the flattened lookups.  Off on
// this path: with the weight floors cutting each row to its admissible prefix, the lookups
// measured faster at every threshold tried (32, 64, 128); the batched form still tunes it.
constexpr uint32_t MERGE_MAX = 0;
// Candidates with more admissible entries than this are spread over many waves.
constexpr uint32_t HEAVY_MIN = 256;

// The weight of (a lower bound of) the M-th heaviest edge, from the load-time histogram.
uint32_t weight_at_rank(const std::vector<uint64_t> &h, uint64_t M) {
    uint64_t cum = 0;
    for (int b = WBINS - 1; b >= 0; b--) {
        cum += h[b];
        if (cum >= M) return weight_bin_low((uint32_t)b);
    }
    return 1;
}

unsigned enum_grid(uint64_t m) {
    const uint64_t chunks = (m + 63) / 64;
    uint64_t blocks = (chunks + 3) / 4;
    const uint64_t cap = (uint64_t)num_cus() * 8;
    if (blocks > cap) blocks = cap;
    return (unsigned)(blocks ? blocks : 1);
}

unsigned filter_grid(uint64_t E) {
    const uint64_t per_block = 256ull * FILTER_UNROLL;
    uint64_t blocks = (E + per_block - 1) / per_block;
    uint64_t cap = (uint64_t)num_cus() * 8;
    if (cap > (uint64_t)MAX_SEG) cap = MAX_SEG;
    if (blocks > cap) blocks = cap;
    return (unsigned)(blocks ? blocks : 1);
}

// Scratch bytes a query holds while it runs (the admission size of a served request).
uint64_t sub_stream_cap(const tt_graph *g, const QueryCtx *q) { return std::min<uint64_t>(q->sub_cap, g->m + 1); }
uint64_t sub_list_cap(const tt_graph *g, const QueryCtx *q) { return std::min<uint64_t>(q->sub_cap, (uint64_t)g->n + 1); }
uint64_t flag_bytes(const tt_graph *g) { return (((uint64_t)g->n + 4) & ~3ull) + 4; }

// Every device block of a context of this query, as the allocator rounds it (an upper bound of
// what the context holds while and after it runs the query), in two parts that each grow with
// one argument: the candidate and triangle buffers (k), and the subset structures (subset_n).
uint64_t query_bytes_k(const tt_graph *g, const QueryCtx *q, uint32_t k) {
    const uint64_t cap = std::max<uint64_t>(q->min_buf, 16ull * k);
    const uint64_t nc = std::min<uint64_t>(g->m + 1, q->max_cand);
    return 2 * dev_round(cap * sizeof(trec)) + dev_round(nc * sizeof(struct cand)) +
           dev_round((uint64_t)std::max<uint32_t>(k, 1) * sizeof(tt_triangle)) + dev_round(MAX_SEG * 4) +
           dev_round(5 * STAT_SLOTS * 8) + dev_round(HEAVY_CAP * sizeof(Heavy)) + dev_round(HEAVY_PIECES * sizeof(uint2)) +
           dev_round(16 * sizeof(unsigned long long)) + dev_round(256);
}
uint64_t query_bytes_sub(const tt_graph *g, const QueryCtx *q, uint32_t subset_n) {
    if (!subset_n) return 0;
    const uint64_t c = (uint64_t)subset_n;
    const uint64_t tmp = ((c * 4 + 7) & ~7ull) + (c + 1) * 4 + 8 + (c + 1) * 8 + WBINS * 8 + c;
    return 2 * dev_round(flag_bytes(g)) + 6 * dev_round(sub_stream_cap(g, q) * 4) + 3 * dev_round(sub_list_cap(g, q) * 4) +
           dev_round(tmp);
}
uint64_t query_bytes(const tt_graph *g, const QueryCtx *q, uint32_t k, uint32_t subset_n) {
    return query_bytes_k(g, q, k) + query_bytes_sub(g, q, subset_n);
}

// Device bytes a context holds now.
uint64_t ctx_bytes(const QueryCtx *q) {
    const void *ptrs[] = {q->buf0, q->buf1, q->cand, q->ccnt, q->spart, q->dcount, q->dout, q->vflag, q->vflag2,
                          q->sub_src, q->sub_col, q->sub_wgt, q->sub_pos, q->sub_vlist, q->sp_c, q->sp_w,
                          q->sp_start, q->sp_cnt, q->heavy, q->nheavy,
                          q->hpiece};
    uint64_t b = 0;
    for (const void *p : ptrs) b += dev_bytes(p);
    return b;
}

} // namespace

int ensure_scratch(const tt_graph *g, QueryCtx *q, uint64_t cap, uint64_t kout) {
    int rc;
    if (q->fixed)
        return q->buf_cap >= cap && q->dout_cap >= kout && q->cand_cap >= 1
                   ? TT_OK
                   : fail(TT_E_TOO_LARGE, "the query needs more scratch than the fixed region holds");
    if (!q->dcount) {
        if ((rc = dev_alloc(nullptr, (void **)&q->dcount, 16 * sizeof(unsigned long long)))) return rc;
        if (hipHostMalloc((void **)&q->hcount, 16 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
            return fail(TT_E_NOMEM, "hipHostMalloc failed");
        for (auto &e : q->ev)
            if (hipEventCreate(&e) != hipSuccess) return fail(TT_E_DEVICE, "hipEventCreate failed");
    }
    if (!q->ccnt && (rc = dev_alloc(nullptr, (void **)&q->ccnt, MAX_SEG * sizeof(uint32_t)))) return rc;
    if (!q->heavy && (rc = dev_alloc(nullptr, (void **)&q->heavy, HEAVY_CAP * sizeof(Heavy)))) return rc;
    if (!q->nheavy && (rc = dev_alloc(nullptr, (void **)&q->nheavy, 256))) return rc;
    if (!q->hpiece && (rc = dev_alloc(nullptr, (void **)&q->hpiece, HEAVY_PIECES * sizeof(uint2)))) return rc;
    if (!q->spart) {
        if ((rc = dev_alloc(nullptr, (void **)&q->spart, 5 * STAT_SLOTS * sizeof(unsigned long long)))) return rc;
        HIP_TRY(hipMemsetAsync(q->spart, 0, 5 * STAT_SLOTS * sizeof(unsigned long long), q->stream));
    }
    const uint64_t cc = std::min<uint64_t>(g->m + 1, q->max_cand);
    if (q->cand_cap < cc) {
        dev_free(nullptr, q->cand, 0);
        q->cand = nullptr;
        q->cand_cap = 0;
        if ((rc = dev_alloc(nullptr, (void **)&q->cand, cc * sizeof(cand)))) return rc;
        q->cand_cap = cc;
    }
    if (q->buf_cap < cap) {
        dev_free(nullptr, q->buf0, 0);
        dev_free(nullptr, q->buf1, 0);
        q->buf0 = q->buf1 = nullptr;
        q->buf_cap = 0;
        if ((rc = dev_alloc(nullptr, (void **)&q->buf0, cap * sizeof(trec))) ||
            (rc = dev_alloc(nullptr, (void **)&q->buf1, cap * sizeof(trec))))
            return rc;
        q->buf_cap = cap;
    }
    if (q->dout_cap < kout) {
        dev_free(nullptr, q->dout, 0);
        if (q->hout) (void)hipHostFree(q->hout);
        q->dout = nullptr;
        q->hout = nullptr;
        q->dout_cap = 0;
        if ((rc = dev_alloc(nullptr, (void **)&q->dout, kout * sizeof(tt_triangle)))) return rc;
        if (hipHostMalloc((void **)&q->hout, kout * sizeof(tt_triangle), hipHostMallocDefault) != hipSuccess) {
            q->hout = nullptr;
            return fail(TT_E_NOMEM, "hipHostMalloc failed");
        }
        q->dout_cap = kout;
    }
    return TT_OK;
}

namespace {

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

// Sorts the first N records of q->buf0 and leaves the best min(N, k) at the front of *res.
int select_topk(QueryCtx *q, uint64_t N, uint32_t k, trec **res) {
    hipStream_t s = q->stream;
    const uint32_t S0 = k < (uint32_t)STILE ? k : (uint32_t)STILE;
    uint64_t nruns = (N + STILE - 1) / STILE;
    trec *in = q->buf0, *out = q->buf1;
    k_tile_sort<<<(unsigned)nruns, 512, 0, s>>>(in, out, N, S0);
    std::swap(in, out);
    uint64_t C = STILE;
    uint32_t S = S0;
    while (nruns > 1) {
        const uint64_t C2 = C * 2;
        const uint32_t So = (uint64_t)k < C2 ? k : (uint32_t)C2;
        const uint64_t nout = (nruns + 1) / 2;
        const uint64_t threads = nout * 2ull * S;
        k_merge<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(in, out, N, C, S, So, nruns);
        std::swap(in, out);
        nruns = nout;
        C = C2;
        S = So;
    }
    HIP_TRY(hipGetLastError());
    *res = in;
    return TT_OK;
}

// Entries to stream for a band with lower key L: every row whose bin is >= bin(score floor).
uint64_t entries_for(const tt_graph *g, int mode, u128 L) {
    const uint64_t t = score_floor(mode, L);
    if (t == 0) return g->m;
    if (t > 0xFFFFFFFFull) return 0;
    const uint32_t b = weight_bin((uint32_t)t);
    return g->ebase[b] + g->ebin[b];
}

struct Stream {
    const uint32_t *src, *col, *wgt, *pos;
    uint64_t E;
    const uint32_t *hmx; // row maximum of each entry's head, or NULL (then gathered)
    uint32_t wbin;       // the weight-ordered stream: the lowest bin it reads; else WBINS
};

// The shortest of the streams that hold every possible base entry of a band triangle: rows
// with hb >= score floor (row order), entries with weight >= weight floor, and (when the
// query has one) entries whose bound reaches the score floor.
// placed_only: the weight-ordered stream is taken only where its bins are already in place.
Stream pick_stream(const tt_graph *g, const BoundOrder *o, int mode, double p, u128 L, bool placed_only = false) {
    Stream r{g->osrc, g->col, g->wgt, nullptr, entries_for(g, mode, L), g->hmx, (uint32_t)WBINS};
    const uint64_t z = weight_floor(mode, p, L, g->wmax);
    if (z > 0xFFFFFFFFull) {
        r.E = 0; // no edge is heavy enough
    } else if (z > 0) {
        const uint32_t b = weight_bin((uint32_t)z);
        const uint64_t E2 = g->wbase[b] + g->whist[b];
        if (E2 < r.E && (!placed_only || g->ws_low.load(std::memory_order_acquire) <= b))
            r = Stream{g->ws_src, g->ws_col, g->ws_wgt, g->ws_pos, E2, g->ws_hmx, b};
    }
    if (o) {
        const uint64_t t = score_floor(mode, L);
        uint64_t E3 = g->m;
        if (t > 0xFFFFFFFFull) E3 = 0;
        else if (t > 0) {
            const uint32_t b = weight_bin((uint32_t)t);
            E3 = o->base[b] + o->hist[b];
        }
        if (E3 < r.E) r = Stream{o->src, o->col, o->wgt, o->pos, E3, nullptr, (uint32_t)WBINS};
    }
    return r;
}

constexpr uint64_t ORDER_AFTER = 4;

tt_graph::StreamedAt &streamed_at(tt_graph *g, uint64_t pb) {
    tt_graph::StreamedAt *lru = &g->streamed[0];
    for (auto &e : g->streamed) {
        if (e.pb == pb && e.last_use) return e;
        if (e.last_use < lru->last_use) lru = &e;
    }
    *lru = tt_graph::StreamedAt();
    lru->pb = pb;
    return *lru;
}

// Records the entries a query of p streamed without a bound order.
void note_streamed(tt_graph *g, double p, uint64_t entries) {
    uint64_t pb;
    std::memcpy(&pb, &p, 8);
    std::lock_guard<std::mutex> lock(g->init_mu);
    tt_graph::StreamedAt &e = streamed_at(g, pb);
    e.entries += entries;
    e.last_use = ++g->order_clock;
}

// The bound order of p for a query; the caller releases it.  It is built once the queries of
// p have streamed more than ORDER_AFTER*m entries through the other orders (so one-off queries
// do not pay for it: on the 2B-edge graph a query without the order takes 71 ms at p = 1 and
// 23 ms at p = +inf, the build ~143 ms).
// Orders of other p are replaced least recently used first, never while a query streams them.
// NULL when there is none (the query then streams the other orders).
int acquire_order(tt_graph *g, QueryCtx *q, double p, BoundOrder **out) {
    *out = nullptr;
    if (g->m == 0) return TT_OK;
    uint64_t pb;
    std::memcpy(&pb, &p, 8);
    BoundOrder *slot = nullptr;
    {
        std::lock_guard<std::mutex> lock(g->init_mu);
        g->order_clock++;
        BoundOrder *empty = nullptr, *lru = nullptr;
        for (uint32_t i = 0; i < g->max_orders; i++) {
            BoundOrder &o = g->bord[i];
            if (o.pb == pb && (o.valid || o.building)) {
                if (!o.valid) return TT_OK; // another query is building it
                o.users++;
                o.last_use = g->order_clock;
                *out = &o;
                return TT_OK;
            }
            if (o.users) continue;
            if (!o.valid) {
                if (!empty) empty = &o;
            } else if (!lru || o.last_use < lru->last_use) {
                lru = &o;
            }
        }
        slot = empty ? empty : lru;
        if (!slot || q->fixed) return TT_OK;
        if (streamed_at(g, pb).entries <= ORDER_AFTER * g->m) return TT_OK;
        // reserved: built below without the lock, so queries of other p are not held up
        slot->valid = false;
        slot->building = true;
        slot->pb = pb;
        slot->users = 1;
    }
    const uint64_t m = g->m;
    hipStream_t s = q->stream;
    unsigned long long *dev = nullptr; // hist | base | cursors
    const int mode = mode_of(p);
    auto body = [&]() -> int {
        int r;
        if (!slot->src && ((r = dev_alloc(g, (void **)&slot->src, (m + 1) * 4)) ||
                           (r = dev_alloc(g, (void **)&slot->col, (m + 1) * 4)) ||
                           (r = dev_alloc(g, (void **)&slot->wgt, (m + 1) * 4)) ||
                           (r = dev_alloc(g, (void **)&slot->pos, (m + 1) * 4))))
            return r;
        if ((r = dev_alloc(nullptr, (void **)&dev, 3 * WBINS * 8))) return r;
        HIP_TRY(hipMemsetAsync(dev, 0, 3 * WBINS * 8, s));
        k_bound_hist<<<enum_grid(m), 256, 0, s>>>(g->osrc, g->col, g->wgt, g->maxw, m, mode, p, dev);
        HIP_TRY(hipGetLastError());
        slot->hist.assign(WBINS, 0);
        HIP_TRY(hipMemcpyAsync(slot->hist.data(), dev, WBINS * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        slot->base.assign(WBINS, 0);
        uint64_t run = 0;
        for (int b = WBINS - 1; b >= 0; b--) { slot->base[b] = run; run += slot->hist[b]; }
        HIP_TRY(hipMemcpyAsync(dev + WBINS, slot->base.data(), WBINS * 8, hipMemcpyHostToDevice, s));
        const unsigned grid = (unsigned)((m + BPLACE_CHUNK - 1) / BPLACE_CHUNK);
        k_place_bound<<<grid, 256, 0, s>>>(g->osrc, g->col, g->wgt, g->maxw, m, mode, p, dev + WBINS,
                                           dev + 2 * WBINS, slot->src, slot->col, slot->wgt, slot->pos);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        return TT_OK;
    };
    int rc = body();
    (void)hipStreamSynchronize(s);
    dev_free(nullptr, dev, 0);
    std::lock_guard<std::mutex> lock(g->init_mu);
    slot->building = false;
    if (rc) {
        slot->users = 0;
        return rc;
    }
    slot->valid = true;
    slot->last_use = ++g->order_clock;
    *out = slot;
    return TT_OK;
}

void release_order(tt_graph *g, BoundOrder *o) {
    if (!o) return;
    std::lock_guard<std::mutex> lock(g->init_mu);
    o->users--;
}

int ensure_band_events(QueryCtx *q, size_t pairs) {
    if (q->fixed) return TT_OK; // no timing
    while (q->band_ev.size() < 2 * pairs) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return fail(TT_E_DEVICE, "hipEventCreate failed");
        q->band_ev.push_back(e);
    }
    return TT_OK;
}

// The filter and intersect kernels of one stream chunk, in the instantiation of the filter
// mode and of the kind of key (generic p or integer).
template <int FILTER, bool GEN> void enqueue_kernels(const EnumArgs &A, unsigned igrid, hipStream_t s) {
    k_filter<FILTER, false, GEN><<<A.nseg, 256, 0, s>>>(A);
    k_intersect<FILTER, false, GEN><<<igrid, 256, 0, s>>>(A);
    k_intersect_heavy<FILTER, false, GEN><<<igrid, 256, 0, s>>>(A);
}

template <bool GEN> void enqueue_pair(int filter, const EnumArgs &A, unsigned igrid, hipStream_t s) {
    if (filter == FILTER_EDGES) enqueue_kernels<FILTER_EDGES, GEN>(A, igrid, s);
    else if (filter == FILTER_VERTICES) enqueue_kernels<FILTER_VERTICES, GEN>(A, igrid, s);
    else enqueue_kernels<FILTER_NONE, GEN>(A, igrid, s);
}

// Enqueues one enumeration pass (no host synchronisation): the band's stream is filtered and
// intersected in pieces of at most cand_cap entries.  `slot` picks its event pair.
int launch_enum(const tt_graph *g, QueryCtx *q, const Band &B, int filter, bool gated, size_t slot) {
    Stream S = q->sub_active ? Stream{q->sub_src, q->sub_col, q->sub_wgt, q->sub_pos, q->sub_len, nullptr, (uint32_t)WBINS}
                             : pick_stream(g, q->ord, B.mode, B.p, B.L, q->fixed);
    if (!q->sub_active && S.wbin < (uint32_t)WBINS && !q->fixed) {
        // the weight-ordered stream: its bins down to S.wbin are placed on first need (lazily
        // built graph state, guarded by the graph's init lock); the stream's arrays are read
        // again after the acquire of ws_low that shows them placed
        if (g->ws_low.load(std::memory_order_acquire) > S.wbin) {
            int rc = ensure_weight_stream(const_cast<tt_graph *>(g), q->stream, S.wbin);
            if (rc) return rc;
        }
        S = pick_stream(g, q->ord, B.mode, B.p, B.L);
    }
    if (S.E && !S.src) return fail(TT_E_DEVICE, "internal: a stream with entries has no arrays");
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
    A.merge_max = MERGE_MAX;
    A.scan_max = SCAN_MAX;
    A.skip = gated ? q->dcount + 7 : nullptr;
    A.B = B;
    A.emark = g->emark;
    A.vflag = q->vflag;
    A.vflag2 = q->vflag2;
    if (q->sub_active) { // the compact subset stream carries the lists of heads in the subset
        A.sp_c = q->sp_c;
        A.sp_w = q->sp_w;
        A.sp_start = q->sp_start;
        A.sp_cnt = q->sp_cnt;
    }
    A.out = q->buf0;
    A.count = q->dcount;
    A.cap = q->buf_cap;
    A.stats = q->spart;
    A.C = q->cand;
    A.ccnt = q->ccnt;
    A.heavy = q->heavy;
    A.nheavy = q->nheavy;
    A.hpiece = q->hpiece;
    A.heavy_min = HEAVY_MIN;
    A.hstat = q->dcount + 12;
    if (!q->fixed) HIP_TRY(hipEventRecord(q->band_ev[2 * slot], q->stream));
    for (uint64_t off = 0; off < S.E; off += q->cand_cap) {
        const uint64_t E = std::min<uint64_t>(S.E - off, q->cand_cap);
        A.s_src = S.src + off;
        A.s_col = S.col + off;
        A.s_wgt = S.wgt + off;
        A.s_pos = S.pos ? S.pos + off : nullptr;
        A.s_hmx = S.hmx ? S.hmx + off : nullptr;
        A.pos_off = off;
        A.E = E;
        A.nseg = filter_grid(E);
        A.seg = (E + A.nseg - 1) / A.nseg;
        const unsigned igrid = (unsigned)num_cus() * 8;
        if (A.B.mode == MODE_GEN) enqueue_pair<true>(filter, A, igrid, q->stream);
        else enqueue_pair<false>(filter, A, igrid, q->stream);
        HIP_TRY(hipGetLastError());
    }
    if (!q->fixed) HIP_TRY(hipEventRecord(q->band_ev[2 * slot + 1], q->stream));
    return TT_OK;
}

// After the stream has been synchronised: add the durations of passes [0, n).
void add_enum_time(QueryCtx *q, tt_query_stats *st, size_t n) {
    if (!st || q->fixed) return;
    for (size_t i = 0; i < n; i++) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, q->band_ev[2 * i], q->band_ev[2 * i + 1]) == hipSuccess) st->enum_kernel_ms += ms;
    }
}

Band make_band(int mode, double p, u128 L, uint32_t Li, uint32_t Lj, uint32_t Ll, bool hasU, u128 U) {
    Band B;
    B.L = L;
    B.Li = Li; B.Lj = Lj; B.Ll = Ll;
    B.U = U;
    B.hasU = hasU ? 1 : 0;
    B.mode = mode;
    B.p = p;
    B.theta = mode == MODE_GEN ? key_as_double(L) : 0.0;
    return B;
}

// Bands are enqueued ahead of the device while they add at most this many pieces (a piece is
// a filter + intersect launch over up to cand_cap stream entries): the late bands of a large
// graph stream most of its entries in many pieces and are rarely needed.
constexpr uint64_t EAGER_PIECES = 8;

uint64_t band_pieces(const tt_graph *g, const QueryCtx *q, const Band &B) {
    const uint64_t E = q->sub_active ? q->sub_len : pick_stream(g, q->ord, B.mode, B.p, B.L, q->fixed).E;
    return std::max<uint64_t>(1, (E + q->cand_cap - 1) / q->cand_cap);
}

// The threshold descent: bands [L_i, L_{i-1}) until >= k triangles are held, restarts on
// overflow, then selection.  Writes min(k, T) triangles to `out` (host).
int run_topk(const tt_graph *g, QueryCtx *q, uint32_t k, double p, int filter, tt_triangle *out, uint32_t *n_out,
             tt_query_stats *st) {
    const int mode = mode_of(p);
    const uint64_t cap = std::max<uint64_t>(q->min_buf, 16ull * k);
    int rc = ensure_scratch(g, q, cap, k);
    if (rc) return rc;
    hipStream_t s = q->stream;
    // Thresholds: L = key(t, t, t) for t = the weight of the M-th heaviest edge (of a subset
    // query's compact stream; with a bound order, the M-th highest entry bound), M = k, 4k,
    // 16k ... while no triangle is found.  Once some are (c < k of them), the next rank is
    // chosen from c: the count above a threshold grows roughly as the cube of the rank on these
    // graphs, so M grows by (4k / c)^(1/3), between 2 and 4, one band at a time.  The last band
    // (L = 0) is exhaustive.
    const std::vector<uint64_t> &hist = q->sub_active ? q->sub_hist : q->ord ? q->ord->hist : g->whist;
    const uint64_t total = q->sub_active ? q->sub_len : g->m;
    // The first rank at or after M (growing by f) whose threshold lies below `below`.  Weights
    // tie in large groups (small integers above all), so the group holding rank M can reach far
    // past it; then the weight bin just above the group is taken when it still lies below
    // `below` (a smaller step than asked for, instead of a much larger one).  Not applied to a
    // bound order's ranks, where it measured slightly slower on the served mix.
    const bool tie_steps = q->ord == nullptr;
    auto next_band = [&](double M, double f, bool has_below, u128 below, double &Mout) -> u128 {
        for (;;) {
            if (M > (double)total) { Mout = (double)total; return 0; }
            uint64_t cum = 0, above = 0; // entries in bins >= b, and in the bins above b
            int b = WBINS - 1, b_up = -1;
            for (; b >= 0; b--) {
                if (hist[b] && cum + hist[b] >= (uint64_t)M) break;
                if (hist[b]) b_up = b;
                cum += hist[b];
            }
            if (b < 0) { Mout = M; return 0; }
            above = cum;
            cum += hist[b];
            if (tie_steps && b_up >= 0 && (double)cum > 2.0 * M) {
                const u128 Lu = key_of_uniform(mode, weight_bin_low((uint32_t)b_up));
                if (!has_below || Lu < below) { Mout = (double)above; return Lu; }
            }
            const uint32_t t = weight_bin_low((uint32_t)b);
            if (t <= 1) { Mout = M; return 0; }
            const u128 L = key_of_uniform(mode, t);
            if (!has_below || L < below) { Mout = M; return L; }
            M *= f;
        }
    };
    HIP_TRY(hipMemsetAsync(q->dcount, 0, 8 * sizeof(unsigned long long), s));
    HIP_TRY(hipMemsetAsync(q->dcount + 12, 0, 2 * sizeof(unsigned long long), s));
    if (!q->fixed) HIP_TRY(hipEventRecord(q->ev[0], s));
    std::vector<u128> Ls;     // thresholds of the bands enqueued, in order
    std::vector<double> Ms;   // their ranks
    size_t launched = 0;      // bands whose events are recorded
    auto enqueue = [&](u128 L, double M, bool gated) -> int {
        const size_t i = Ls.size();
        int r = ensure_band_events(q, launched + 1);
        if (r) return r;
        if (gated) {
            k_band_gate<<<1, 64, 0, s>>>(q->dcount, 1ull, q->dcount + 7, (unsigned long long)i, q->dcount + 6);
            HIP_TRY(hipGetLastError());
        }
        const Band B = make_band(mode, p, L, ~0u, ~0u, ~0u, i > 0, i > 0 ? Ls.back() : 0);
        if ((r = launch_enum(g, q, B, filter, gated, launched))) return r;
        Ls.push_back(L);
        Ms.push_back(M);
        launched++;
        return TT_OK;
    };
    auto read_count = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(q->hcount, q->dcount, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return TT_OK;
    };
    {
        double M0;
        const u128 L0 = next_band((double)k, 4.0, false, 0, M0);
        if ((rc = enqueue(L0, M0, false)) || (rc = read_count())) return rc;
    }
    // The first band often holds the whole answer, so the host reads the count after it.
    // While the count is zero, later bands (x4 in rank) are enqueued without waiting while
    // their pieces fit EAGER_PIECES; the gate before each stops the rest once the buffer holds
    // any triangle and records the last band that ran.
    size_t last = 0; // index of the last band that ran
    while (q->hcount[0] < k && Ls.back() != 0) {
        const uint64_t c = q->hcount[0];
        if (c == 0) {
            uint64_t pending = 0;
            double M = Ms[last] * 4.0;
            while (Ls.back() != 0) {
                double Mn;
                const u128 L = next_band(M, 4.0, true, Ls.back(), Mn);
                const Band B = make_band(mode, p, L, ~0u, ~0u, ~0u, true, Ls.back());
                const uint64_t np = band_pieces(g, q, B);
                if (pending > 0 && pending + np > EAGER_PIECES) break;
                if ((rc = enqueue(L, Mn, true))) return rc;
                pending += np;
                M = Mn * 4.0;
            }
            if ((rc = read_count())) return rc;
            last = q->hcount[7] ? (size_t)q->hcount[6] : Ls.size() - 1;
            if (q->hcount[0] >= k) break;
            // paused after the first band with triangles: drop the bands that did not run (the
            // bands from here on are not gated, so the skip flag stays as it is)
            Ls.resize(last + 1);
            Ms.resize(last + 1);
        } else {
            const double f = std::min(4.0, std::max(2.0, std::cbrt(4.0 * (double)k / (double)c)));
            double Mn;
            const u128 L = next_band(Ms[last] * f, f, true, Ls.back(), Mn);
            if ((rc = enqueue(L, Mn, false)) || (rc = read_count())) return rc;
            last = Ls.size() - 1;
        }
    }
    add_enum_time(q, st, launched);
    uint64_t cnt = q->hcount[0];
    bool overflow = cnt > q->buf_cap;
    double sel_ms = 0.0;
    while (overflow) {
        // the k-th best of the records kept is a lower bound on the k-th best overall
        trec *res = nullptr;
        if (!q->fixed) HIP_TRY(hipEventRecord(q->ev[2], s));
        if ((rc = select_topk(q, q->buf_cap, k, &res))) return rc;
        trec kth;
        HIP_TRY(hipMemcpyAsync(&kth, res + (k - 1), sizeof(trec), hipMemcpyDeviceToHost, s));
        if (!q->fixed) HIP_TRY(hipEventRecord(q->ev[3], s));
        HIP_TRY(hipMemsetAsync(q->dcount, 0, sizeof(unsigned long long), s));
        HIP_TRY(hipStreamSynchronize(s));
        float ms = 0.f;
        if (!q->fixed) (void)hipEventElapsedTime(&ms, q->ev[2], q->ev[3]);
        sel_ms += ms;
        const u128 L = ((u128)kth.khi << 64) | kth.klo;
        rc = launch_enum(g, q, make_band(mode, p, L, kth.i, kth.j, kth.l, false, 0), filter, false, 0);
        if (rc) return rc;
        if (st) st->restarts++;
        HIP_TRY(hipMemcpyAsync(q->hcount, q->dcount, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        add_enum_time(q, st, 1);
        cnt = q->hcount[0];
        overflow = cnt > q->buf_cap;
    }
    if (!q->fixed) HIP_TRY(hipEventRecord(q->ev[1], s));
    const uint64_t N = cnt;
    const uint32_t K = (uint32_t)std::min<uint64_t>(N, k);
    if (K > 0) {
        trec *res = nullptr;
        if ((rc = select_topk(q, N, k, &res))) return rc;
        k_finalize<<<(K + 255) / 256, 256, 0, s>>>(res, K, mode, q->dout);
        HIP_TRY(hipGetLastError());
    }
    if (!q->fixed) HIP_TRY(hipEventRecord(q->ev[2], s));
    k_reduce_stats<<<5, 256, 0, s>>>(q->spart, q->dcount + 1);
    // results through pinned staging (the caller's buffer is ordinary host memory; a fixed
    // context copies straight to it), counters in one copy
    if (K > 0)
        HIP_TRY(hipMemcpyAsync(q->fixed ? (void *)out : (void *)q->hout, q->dout, (size_t)K * sizeof(tt_triangle),
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(q->hcount, q->dcount, 16 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (K > 0 && !q->fixed) std::memcpy(out, q->hout, (size_t)K * sizeof(tt_triangle));
    *n_out = K;
    if (st) {
        float e_ms = 0.f, s_ms = 0.f;
        if (!q->fixed) {
            (void)hipEventElapsedTime(&e_ms, q->ev[0], q->ev[1]);
            (void)hipEventElapsedTime(&s_ms, q->ev[1], q->ev[2]);
        }
        st->enum_ms += e_ms;
        st->select_ms += s_ms + sel_ms;
        st->candidate_edges += q->hcount[1];
        st->intersected_entries += q->hcount[2];
        st->triangles_emitted += q->hcount[3];
        st->edges_streamed += q->hcount[4];
        st->passes += (uint32_t)q->hcount[5];
        st->heavy_candidates += q->hcount[12];
        st->heavy_overflow += q->hcount[13];
    }
    return TT_OK;
}

} // namespace

// The first N records of q->buf0 sorted, the best min(N, k) at the front of *res.
int select_records(QueryCtx *q, uint64_t N, uint32_t k, trec **res) { return select_topk(q, N, k, res); }

// Selection of the first N records of q->buf0 (the candidate triangles of a query that found
// them by other means, e.g. a sampler): the best min(N, k), finalised and copied to `out`.
int finish_topk(QueryCtx *q, uint64_t N, uint32_t k, int mode, tt_triangle *out, uint32_t *n_out) {
    hipStream_t s = q->stream;
    const uint32_t K = (uint32_t)std::min<uint64_t>(N, k);
    *n_out = 0;
    if (K == 0) return TT_OK;
    trec *res = nullptr;
    int rc = select_topk(q, N, k, &res);
    if (rc) return rc;
    k_finalize<<<(K + 255) / 256, 256, 0, s>>>(res, K, mode, q->dout);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(q->hout, q->dout, (size_t)K * sizeof(tt_triangle), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(out, q->hout, (size_t)K * sizeof(tt_triangle));
    *n_out = K;
    return TT_OK;
}

namespace {

int ensure_flags(const tt_graph *g, QueryCtx *q) {
    int rc;
    if (!q->vflag && (rc = dev_alloc(nullptr, (void **)&q->vflag, flag_bytes(g)))) return rc;
    if (!q->vflag2 && (rc = dev_alloc(nullptr, (void **)&q->vflag2, flag_bytes(g)))) return rc;
    return TT_OK;
}

int check_query(const tt_graph *g, double p, const tt_triangle *out, uint32_t k, uint32_t *n_out) {
    if (n_out) *n_out = 0;
    if (!g) return fail(TT_E_ARG, "graph is NULL");
    if (!n_out) return fail(TT_E_ARG, "n_out is NULL");
    if (std::isnan(p)) return fail(TT_E_ARG, "p is NaN");
    if (k && !out) return fail(TT_E_ARG, "out is NULL");
    return TT_OK;
}

int check_subset(const tt_graph *g, const uint32_t *subset, uint32_t subset_n) {
    for (uint32_t t = 0; subset && t < subset_n; t++)
        if (subset[t] >= g->n) return fail(TT_E_VERTEX_RANGE, "subset vertex >= n");
    return TT_OK;
}

// Marks the subset (vflag) and the vertices with an out-neighbour in it (vflag2), then builds
// the compact stream of the entries that can be the base of a triangle touching the subset.
// If the stream or the list would not fit (huge subsets), the passes stream every entry with
// the vertex pre-tests instead.
constexpr uint64_t SUB_SCAN_MUL = 8;

int prepare_subset(tt_graph *g, QueryCtx *q, const uint32_t *subset, uint32_t cnt) {
    int rc;
    q->sub_active = false;
    if ((rc = ensure_in_csr(g, q->stream)) || (rc = ensure_flags(g, q))) return rc;
    const uint64_t scap = sub_stream_cap(g, q), vcap = sub_list_cap(g, q);
    if (!q->sub_src) {
        if ((rc = dev_alloc(nullptr, (void **)&q->sub_src, scap * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&q->sub_col, scap * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&q->sub_wgt, scap * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&q->sub_pos, scap * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&q->sub_vlist, vcap * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&q->sp_c, scap * 4)) || (rc = dev_alloc(nullptr, (void **)&q->sp_w, scap * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&q->sp_start, vcap * 4)) ||
            (rc = dev_alloc(nullptr, (void **)&q->sp_cnt, vcap * 4)))
            return rc;
    }
    // per-query scratch: ids[cnt] | lens[cnt+1] | pre[cnt+1] (u64) | hist[WBINS] (u64) | own[cnt]
    const uint64_t o_lens = ((uint64_t)cnt * 4 + 7) & ~7ull, o_pre = (o_lens + ((uint64_t)cnt + 1) * 4 + 7) & ~7ull;
    const uint64_t o_hist = o_pre + ((uint64_t)cnt + 1) * 8, o_own = o_hist + WBINS * 8;
    const uint64_t bytes = o_own + cnt;
    char *tmp = nullptr;
    if ((rc = dev_alloc(nullptr, (void **)&tmp, bytes))) return rc;
    uint32_t *ids = (uint32_t *)tmp, *lens = (uint32_t *)(tmp + o_lens);
    uint64_t *pre = (uint64_t *)(tmp + o_pre);
    unsigned long long *hist = (unsigned long long *)(tmp + o_hist);
    uint8_t *own = (uint8_t *)(tmp + o_own);
    unsigned long long *cnt8 = q->dcount + 8; // [0] listed in-neighbours [1] row entries [2] kept
    hipStream_t s = q->stream;
    auto body = [&]() -> int {
        HIP_TRY(hipMemsetAsync(q->vflag, 0, flag_bytes(g), s));
        HIP_TRY(hipMemsetAsync(q->vflag2, 0, flag_bytes(g), s));
        HIP_TRY(hipMemsetAsync(cnt8, 0, 4 * sizeof(unsigned long long), s));
        HIP_TRY(hipMemsetAsync(hist, 0, WBINS * 8, s));
        HIP_TRY(hipMemcpyAsync(ids, subset, (uint64_t)cnt * 4, hipMemcpyHostToDevice, s));
        k_sub_mark<<<(cnt + 1 + 255) / 256, 256, 0, s>>>(ids, cnt, g->irstart, g->rlen, q->vflag, own, lens, cnt8);
        HIP_TRY(hipGetLastError());
        if ((rc = exclusive_scan_u32_to_u64(lens, pre, (uint64_t)cnt + 1, s, nullptr))) return rc;
        k_sub_in<<<num_cus() * 8, 256, 0, s>>>(ids, cnt, pre, g->irstart, g->itail, g->rlen, q->vflag, q->vflag2,
                                               q->sub_vlist, vcap, cnt8);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(q->hcount + 8, cnt8, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        // The rows to scan bound the compact stream; most of their entries are usually dropped
        // (a subset vertex of high in-degree lists many in-neighbours whose rows lead elsewhere),
        // so rows up to SUB_SCAN_MUL times the capacity are scanned, and the stream is used if
        // the entries kept fit.  Otherwise: the full stream with vertex pre-tests.
        const uint64_t nv = q->hcount[8], bound = q->hcount[9];
        if (nv > vcap || bound > SUB_SCAN_MUL * scap) return TT_OK;
        k_sub_rows<<<num_cus() * 8, 256, 0, s>>>(ids, own, cnt, q->sub_vlist, (uint32_t)nv, g->rstart, g->rlen,
                                                 g->col, g->wgt, q->vflag, q->vflag2, q->sub_src, q->sub_col,
                                                 q->sub_wgt, q->sub_pos, scap, q->sp_c, q->sp_w, q->sp_start,
                                                 q->sp_cnt, cnt8, hist);
        HIP_TRY(hipGetLastError());
        q->sub_hist.assign(WBINS, 0);
        HIP_TRY(hipMemcpyAsync(q->sub_hist.data(), hist, WBINS * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(q->hcount + 10, cnt8 + 2, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        q->sub_len = q->hcount[10];
        q->sub_active = q->sub_len <= scap; // else some kept entries did not fit: full stream
        return TT_OK;
    };
    rc = body();
    (void)hipStreamSynchronize(s);
    dev_free(nullptr, tmp, bytes);
    return rc;
}

// One exact query on context q (the caller serialises use of q).
int query_on(tt_graph *g, QueryCtx *q, uint32_t k, double p, const uint32_t *subset, uint32_t subset_n,
             tt_triangle *out, uint32_t *n_out, tt_query_stats *stats) {
    int filter = FILTER_NONE, rc;
    q->sub_active = false;
    if (subset && subset_n) {
        if ((rc = ensure_scratch(g, q, std::max<uint64_t>(q->min_buf, 16ull * k), k)) ||
            (rc = prepare_subset(g, q, subset, subset_n)))
            return rc;
        filter = FILTER_VERTICES;
    }
    BoundOrder *o = nullptr;
    if (!q->sub_active && (rc = acquire_order(g, q, p, &o))) return rc;
    q->ord = o;
    if (stats) stats->bound_order = o ? 1 : 0;
    rc = run_topk(g, q, k, p, filter, out, n_out, stats);
    q->ord = nullptr;
    release_order(g, o);
    if (!rc && !o && !q->sub_active) note_streamed(g, p, q->hcount[4]);
    q->sub_active = false;
    return rc;
}

// Prefix sums of w^q (input order) and their guide table, for the two most recent q.
int sample_table(tt_graph *g, double qexp, int kind, tt_graph::SampleTable **out) {
    g->use_clock++;
    for (auto &t : g->tables)
        if (t.q == qexp && t.prefix) { t.last_use = g->use_clock; *out = &t; return TT_OK; }
    tt_graph::SampleTable *t = &g->tables[0];
    if (g->tables[1].last_use < t->last_use) t = &g->tables[1];
    int rc;
    if (!g->guide_bits) {
        uint32_t bits = 1;
        while (bits < 26 && (1ull << (bits + 1)) <= g->m) bits++;
        g->guide_bits = bits;
    }
    if (!t->prefix && (rc = dev_alloc(g, &t->prefix, g->m * 16))) return rc;
    if (!t->scan_tmp && (rc = dev_alloc(g, &t->scan_tmp, scan_tmp_bytes(g->m)))) return rc;
    if (!t->guide && (rc = dev_alloc(g, (void **)&t->guide, ((1ull << g->guide_bits) + 1) * 4))) return rc;
    t->q = -1.0;
    if ((rc = inclusive_weight_prefix(g, qexp, t->prefix, t->scan_tmp))) return rc; // enqueued only
    const uint64_t runs = ((1ull << g->guide_bits) + GUIDE_RUN - 1) / GUIDE_RUN + 1;
    const unsigned grid = (unsigned)std::min<uint64_t>((runs + 255) / 256, (uint64_t)num_cus() * 16);
    if (kind == 0) k_es_guide<0><<<grid, 256, 0, g->stream>>>(t->prefix, g->m, g->guide_bits, t->guide);
    else if (kind == 1) k_es_guide<1><<<grid, 256, 0, g->stream>>>(t->prefix, g->m, g->guide_bits, t->guide);
    else k_es_guide<2><<<grid, 256, 0, g->stream>>>(t->prefix, g->m, g->guide_bits, t->guide);
    HIP_TRY(hipGetLastError());
    t->q = qexp;
    t->last_use = g->use_clock;
    *out = t;
    return TT_OK;
}

} // namespace

extern "C" int topk_triangles_ex(tt_graph *g, uint32_t k, double p, const uint32_t *subset, uint32_t subset_n,
                                 tt_triangle *out, uint32_t *n_out, tt_query_stats *stats) {
    Timer timer;
    int rc = check_query(g, p, out, k, n_out);
    if (rc) return rc;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if ((rc = check_subset(g, subset, subset_n))) return rc;
    if (k == 0 || g->m == 0) { set_error(""); return TT_OK; }
    std::lock_guard<std::mutex> lock(g->mu);
    (void)hipSetDevice(g->device);
    rc = query_on(g, &g->q, k, p, subset, subset_n, out, n_out, stats);
    if (stats) stats->total_ms = timer.ms();
    if (!rc) set_error("");
    return rc;
}

extern "C" int topk_triangles(tt_graph *g, uint32_t k, double p, tt_triangle *out, uint32_t *n_out) {
    return topk_triangles_ex(g, k, p, nullptr, 0, out, n_out, nullptr);
}

extern "C" int sample_heavy_triangles_ex(tt_graph *g, uint32_t k, double p, uint64_t budget, uint64_t seed,
                                         double qexp, uint32_t *draws, tt_triangle *out, uint32_t *n_out,
                                         tt_query_stats *stats) {
    Timer timer;
    int rc = check_query(g, p, out, k, n_out);
    if (rc) return rc;
    if (!std::isnan(qexp) && !(qexp > 0.0 && std::isfinite(qexp)))
        return fail(TT_E_ARG, "the sampling exponent q must be finite and > 0 (or NaN for the default)");
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (budget == 0 || g->m == 0 || (k == 0 && !draws)) { set_error(""); return TT_OK; }
    std::lock_guard<std::mutex> lock(g->mu);
    (void)hipSetDevice(g->device);
    QueryCtx *q = &g->q;
    if ((rc = ensure_flags(g, q)) || (rc = ensure_scratch(g, q, 1, 1))) return rc;
    if (!g->emark && (rc = dev_alloc(g, (void **)&g->emark, g->m + 1))) return rc;
    if ((rc = ensure_opos(g, q->stream))) return rc;
    if (std::isnan(qexp)) qexp = (std::isfinite(p) && p > 0.0) ? p : 1.0;
    const int kind = qexp == 1.0 ? 0 : (qexp == 2.0 || qexp == 3.0) ? 1 : 2;
    hipStream_t s = q->stream;
    uint32_t *ddump = nullptr; // device copy of the draw sequence (draws != NULL)
    if (draws && (rc = dev_alloc(nullptr, (void **)&ddump, budget * 4))) return rc;
    struct DumpGuard { // returned to the cache once the stream is done with it
        uint32_t *p; hipStream_t s;
        ~DumpGuard() { if (p) { (void)hipStreamSynchronize(s); dev_free(nullptr, p, 0); } }
    } dump_guard{ddump, s};
    HIP_TRY(hipEventRecord(q->ev[6], s));
    tt_graph::SampleTable *tab = nullptr;
    if ((rc = sample_table(g, qexp, kind, &tab))) return rc;
    HIP_TRY(hipMemsetAsync(g->emark, 0, g->m + 1, s));
    HIP_TRY(hipMemsetAsync(q->vflag, 0, (uint64_t)g->n + 1, s));
    HIP_TRY(hipMemsetAsync(q->dcount + 14, 0, sizeof(unsigned long long), s)); // distinct draws
    const unsigned grid = (unsigned)std::min<uint64_t>((budget + 255) / 256, (uint64_t)num_cus() * 16);
    const uint32_t bits = g->guide_bits;
    if (kind == 0) k_es_draw<0><<<grid, 256, 0, s>>>(tab->prefix, tab->guide, bits, g->m, budget, seed, g->opos, g->emark, ddump);
    else if (kind == 1) k_es_draw<1><<<grid, 256, 0, s>>>(tab->prefix, tab->guide, bits, g->m, budget, seed, g->opos, g->emark, ddump);
    else k_es_draw<2><<<grid, 256, 0, s>>>(tab->prefix, tab->guide, bits, g->m, budget, seed, g->opos, g->emark, ddump);
    k_mark_tails<<<enum_grid(g->m / 16 + 1), 256, 0, s>>>(g->emark, g->m, g->osrc, q->vflag, q->dcount + 14);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(q->ev[7], s));
    if (ddump) {
        HIP_TRY(hipMemcpyAsync(draws, ddump, budget * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (k == 0) {
            if (stats) stats->total_ms = timer.ms();
            set_error("");
            return TT_OK;
        }
    }
    BoundOrder *o = nullptr;
    if ((rc = acquire_order(g, q, p, &o))) return rc;
    q->ord = o;
    if (stats) stats->bound_order = o ? 1 : 0;
    rc = run_topk(g, q, k, p, FILTER_EDGES, out, n_out, stats);
    q->ord = nullptr;
    release_order(g, o);
    if (!rc && !o) note_streamed(g, p, q->hcount[4]);
    if (!rc && stats) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, q->ev[6], q->ev[7]) == hipSuccess) stats->sample_ms = ms;
        stats->distinct_sampled = q->hcount[14]; // counted by k_mark_tails, copied with the counters
        stats->total_ms = timer.ms();
    }
    if (!rc) set_error("");
    return rc;
}

extern "C" int sample_heavy_triangles(tt_graph *g, uint32_t k, double p, uint64_t budget, uint64_t seed,
                                      tt_triangle *out, uint32_t *n_out) {
    return sample_heavy_triangles_ex(g, k, p, budget, seed, __builtin_nan(""), nullptr, out, n_out, nullptr);
}

// Alg. 3's draws for the clique sampler: g->emark marks the head-sorted entry of every edge drawn
// in `budget` draws with exponent qexp (the draw rule of sample_heavy_triangles).  The caller
// holds g->mu; the work is enqueued on q->stream.
int es_mark_edges(tt_graph *g, QueryCtx *q, double qexp, uint64_t budget, uint64_t seed) {
    int rc;
    if (!g->emark && (rc = dev_alloc(g, (void **)&g->emark, g->m + 1))) return rc;
    if ((rc = ensure_opos(g, q->stream))) return rc;
    const int kind = qexp == 1.0 ? 0 : (qexp == 2.0 || qexp == 3.0) ? 1 : 2;
    hipStream_t s = q->stream;
    tt_graph::SampleTable *tab = nullptr;
    if ((rc = sample_table(g, qexp, kind, &tab))) return rc;
    HIP_TRY(hipMemsetAsync(g->emark, 0, g->m + 1, s));
    const unsigned grid = (unsigned)std::min<uint64_t>((budget + 255) / 256, (uint64_t)num_cus() * 16);
    const uint32_t bits = g->guide_bits;
    if (kind == 0) k_es_draw<0><<<grid, 256, 0, s>>>(tab->prefix, tab->guide, bits, g->m, budget, seed, g->opos, g->emark, nullptr);
    else if (kind == 1) k_es_draw<1><<<grid, 256, 0, s>>>(tab->prefix, tab->guide, bits, g->m, budget, seed, g->opos, g->emark, nullptr);
    else k_es_draw<2><<<grid, 256, 0, s>>>(tab->prefix, tab->guide, bits, g->m, budget, seed, g->opos, g->emark, nullptr);
    HIP_TRY(hipGetLastError());
    return TT_OK;
}

// ----------------------------------------------------------------------------- no allocation
// topk_triangles_noalloc: topk_triangles with its device scratch in one static array per
// device (`scratch`), for callers that cannot allocate.  The array's device address is taken
// once per device with hipGetSymbolAddress; the host-side name is never used as an address.
namespace {
constexpr uint64_t NOALLOC_BYTES = 64ull << 20;
constexpr uint32_t NOALLOC_MAX_K = 16384;
constexpr uint64_t NOALLOC_BUF = 16ull * NOALLOC_MAX_K; // triangle records per buffer
constexpr int NOALLOC_DEVICES = 64;
} // namespace

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
struct NoAllocDevice {
    std::mutex mu;                  // one call at a time per device
    unsigned char *base = nullptr;  // device address of this device's `scratch`
    QueryCtx q;                     // its fields point into `scratch` (q.fixed)
    unsigned long long hcount[16] = {};
};
NoAllocDevice g_noalloc[NOALLOC_DEVICES];

// With the device current: the array's address and the query context carved from it.
int noalloc_setup(NoAllocDevice &D) {
    void *addr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !addr)
        return fail(TT_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    unsigned char *base = (unsigned char *)addr;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        void *r = base + off;
        off += (bytes + 255) & ~255ull;
        return r;
    };
    QueryCtx &q = D.q;
    q.fixed = true;
    q.dcount = (unsigned long long *)take(16 * sizeof(unsigned long long));
    q.spart = (unsigned long long *)take(5 * STAT_SLOTS * sizeof(unsigned long long));
    q.ccnt = (uint32_t *)take(MAX_SEG * sizeof(uint32_t));
    q.nheavy = (unsigned long long *)take(256);
    q.heavy = (Heavy *)take(HEAVY_CAP * sizeof(Heavy));
    q.hpiece = (uint2 *)take(HEAVY_PIECES * sizeof(uint2));
    q.dout = (tt_triangle *)take(NOALLOC_MAX_K * sizeof(tt_triangle));
    q.dout_cap = NOALLOC_MAX_K;
    q.buf0 = (trec *)take(NOALLOC_BUF * sizeof(trec));
    q.buf1 = (trec *)take(NOALLOC_BUF * sizeof(trec));
    q.buf_cap = q.min_buf = NOALLOC_BUF;
    q.cand = (cand *)(base + off); // the rest: candidate entries of a piece of a pass
    q.cand_cap = q.max_cand = (NOALLOC_BYTES - off) / sizeof(cand);
    q.hcount = D.hcount;
    D.base = base;
    return TT_OK;
}
} // namespace

extern "C" int topk_triangles_noalloc(tt_graph *g, uint32_t k, double p, tt_triangle *out, uint32_t *n_out) {
    static_assert(NOALLOC_BYTES >= (16ull << 20) + 2 * NOALLOC_BUF * sizeof(trec) + 2 * HEAVY_CAP * sizeof(Heavy),
                  "the fixed region leaves room for a candidate list");
    int rc = check_query(g, p, out, k, n_out);
    if (rc) return rc;
    if (k > NOALLOC_MAX_K) return fail(TT_E_TOO_LARGE, "topk_triangles_noalloc: k must be <= 16384");
    if (k == 0 || g->m == 0) { set_error(""); return TT_OK; }
    if (g->device < 0 || g->device >= NOALLOC_DEVICES) return fail(TT_E_DEVICE, "device ordinal beyond 63");
    NoAllocDevice &D = g_noalloc[g->device];
    std::lock_guard<std::mutex> dlock(D.mu);
    std::lock_guard<std::mutex> glock(g->mu);
    (void)hipSetDevice(g->device);
    if (!D.base && (rc = noalloc_setup(D))) return rc;
    QueryCtx *q = &D.q;
    q->stream = g->stream;
    // the array keeps the previous call's contents: the spread counters start at zero (the
    // other counters are cleared by the query itself)
    HIP_TRY(hipMemsetAsync(q->spart, 0, 5 * STAT_SLOTS * sizeof(unsigned long long), q->stream));
    BoundOrder *o = nullptr;
    if ((rc = acquire_order(g, q, p, &o))) return rc; // an order already built, never a new one
    q->ord = o;
    rc = run_topk(g, q, k, p, FILTER_NONE, out, n_out, nullptr);
    q->ord = nullptr;
    release_order(g, o);
    if (!rc) set_error("");
    return rc;
}

// ----------------------------------------------------------------------------- serving
// A request loop over one resident graph.  Each slot is a worker thread with its own query
// context and HIP stream, so admitted requests overlap on the device.  Requests wait in FIFO
// order and are admitted as soon as a slot is free and their scratch bytes fit the budget
// (continuous batching: a request that arrives while others run starts when one finishes).
struct tt_server {
    ServeCore core;
    tt_graph *g = nullptr;
    std::vector<QueryCtx> ctx;
    std::vector<std::thread> workers;
};

extern "C" int server_create(tt_graph *g, uint32_t slots, uint64_t scratch_budget, tt_server **out) {
    if (!out) return fail(TT_E_ARG, "out is NULL");
    *out = nullptr;
    if (!g || slots == 0 || slots > 64) return fail(TT_E_ARG, "graph is NULL or slots not in [1, 64]");
    tt_server *S = new (std::nothrow) tt_server();
    if (!S) return fail(TT_E_NOMEM, "host allocation failed");
    S->g = g;
    S->core.budget = scratch_budget;
    S->core.held.assign(slots, ServeCore::Parts{});
    S->core.actual.assign(slots, 0);
    S->ctx.resize(slots);
    for (auto &q : S->ctx) {
        q.min_buf = 1ull << 20;
        q.max_cand = 1ull << 24;
        if (hipStreamCreateWithFlags(&q.stream, hipStreamNonBlocking) != hipSuccess) {
            for (auto &c : S->ctx)
                if (c.stream) (void)hipStreamDestroy(c.stream);
            delete S;
            return fail(TT_E_DEVICE, "hipStreamCreate failed");
        }
        q.owns_stream = true;
    }
    for (size_t i = 0; i < slots; i++)
        S->workers.emplace_back([S, i] {
            QueryCtx *q = &S->ctx[i];
            (void)hipSetDevice(S->g->device);
            S->core.worker(
                i,
                [&](const ServeCore::Req &r, ServeCore::Res &res) -> uint64_t {
                    res.rc = query_on(S->g, q, r.k, r.p, r.subset.empty() ? nullptr : r.subset.data(),
                                      (uint32_t)r.subset.size(), res.tri.data(), &res.n_out, &res.st);
                    if (res.rc) res.err = tt_last_error();
                    // the slot keeps its scratch for the next request (it only grows with k)
                    return ctx_bytes(q);
                },
                [&] { ctx_release(q); });
        });
    *out = S;
    set_error("");
    return TT_OK;
}

extern "C" uint64_t server_request_bytes(tt_server *S, uint32_t k, uint32_t subset_n) {
    if (!S) return 0;
    return query_bytes(S->g, &S->ctx[0], k, subset_n);
}

extern "C" int server_submit(tt_server *S, uint32_t k, double p, const uint32_t *subset, uint32_t subset_n,
                             uint64_t *ticket) {
    if (!S || !ticket) return fail(TT_E_ARG, "server or ticket is NULL");
    *ticket = 0;
    if (std::isnan(p)) return fail(TT_E_ARG, "p is NaN");
    int rc = check_subset(S->g, subset, subset_n);
    if (rc) return rc;
    ServeCore::Req r;
    r.k = k;
    r.p = p;
    if (subset && subset_n) r.subset.assign(subset, subset + subset_n);
    r.need[0] = query_bytes_k(S->g, &S->ctx[0], k);
    r.need[1] = query_bytes_sub(S->g, &S->ctx[0], (uint32_t)r.subset.size());
    rc = S->core.submit(std::move(r), ticket);
    if (rc == TT_E_BUDGET) return fail(rc, "the request needs more scratch than the server's budget");
    if (rc) return fail(rc, "server is shutting down");
    set_error("");
    return TT_OK;
}

extern "C" int server_poll(tt_server *S, uint64_t ticket, int *done) {
    if (!S || !done) return fail(TT_E_ARG, "server or done is NULL");
    if (S->core.poll(ticket, done)) return fail(TT_E_ARG, "unknown ticket");
    return TT_OK;
}

extern "C" int server_wait(tt_server *S, uint64_t ticket, tt_triangle *out, uint32_t *n_out, tt_query_stats *stats) {
    if (n_out) *n_out = 0;
    if (!S || !n_out) return fail(TT_E_ARG, "server or n_out is NULL");
    ServeCore::Res res;
    if (S->core.wait(ticket, res)) return fail(TT_E_ARG, "unknown ticket");
    if (res.rc) return fail(res.rc, res.err);
    if (res.n_out && !out) return fail(TT_E_ARG, "out is NULL");
    std::memcpy(out, res.tri.data(), (size_t)res.n_out * sizeof(tt_triangle));
    *n_out = res.n_out;
    if (stats) *stats = res.st;
    set_error("");
    return TT_OK;
}

extern "C" uint64_t server_scratch_bytes(tt_server *S) { return S ? S->core.held_bytes() : 0; }

extern "C" int server_info(tt_server *S, uint64_t *admitted, uint64_t *completed, uint64_t *peak_bytes,
                           uint32_t *max_queue, uint32_t *max_running) {
    if (!S) return fail(TT_E_ARG, "server is NULL");
    ServeCore &C = S->core;
    std::lock_guard<std::mutex> lk(C.mu);
    if (admitted) *admitted = C.admitted;
    if (completed) *completed = C.completed;
    if (peak_bytes) *peak_bytes = C.peak;
    if (max_queue) *max_queue = C.max_queue;
    if (max_running) *max_running = C.max_running;
    return TT_OK;
}

extern "C" void server_destroy(tt_server *S) {
    if (!S) return;
    S->core.shutdown();
    for (auto &t : S->workers) t.join();
    for (auto &q : S->ctx) {
        ctx_release(&q);
        if (q.owns_stream && q.stream) (void)hipStreamDestroy(q.stream);
    }
    delete S;
}
