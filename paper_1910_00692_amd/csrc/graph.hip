// graph.hip — graph_load: validation and the degree-oriented CSR, built on the device.
//
// The brute-force enumerator of Sec. 3 (NodeIterator++) visits each triangle once from its
// vertex of highest degree; the equivalent edge view used here orients every edge from the
// endpoint that is lower in (degree, ID) order to the higher one, so that each triangle
// {a < b < c} (in that order) is found exactly once, at entry a->b, as c in out(a) ∩ out(b).
// Out-degrees are then at most sqrt(2m), which bounds the cost of every intersection.
//
// Row bound and layout.  A triangle based at u has two edges in u's out-row and one in the
// out-row of an out-neighbour v, so its score, for every p, is at most
// hb[u] = max(maxw[u], max over v of maxw[v]) (m_p never exceeds the largest weight).  Rows
// are stored grouped by weight_bin(hb) in descending order; a pass that only needs triangles
// of score >= t then streams a prefix of the entry arrays.  Each row is also kept sorted by
// weight (descending) so that the entries at or above a weight floor form a prefix.
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <map>
#include <unordered_map>

#include "common.h"

// ----------------------------------------------------------------------------- errors
static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}
extern "C" const char *tt_last_error(void) { return g_last_error.c_str(); }

// Device memory comes from a process-wide cache of freed blocks (exact rounded sizes, per
// device), so that repeated loads and queries do not pay for hipMalloc/hipFree: returning a large
// block to the driver and asking for it again costs far more than the work that uses it.  The
// cache holds up to 3/4 of each device's memory; tt_trim_cache() hands it all back.  Blocks are
// only returned to the cache after the work that used them has completed on its stream.
namespace {
struct Block {
    size_t size;
    int device;
};
std::mutex g_pool_mu;
std::multimap<std::pair<int, size_t>, void *> g_pool;  // free blocks by (device, size)
std::unordered_map<void *, Block> g_live;             // every block handed out
std::unordered_map<int, size_t> g_pool_bytes;         // cached bytes per device
std::unordered_map<int, size_t> g_pool_cap;           // cache limit per device

size_t round_size(size_t b) {
    if (b == 0) b = 16;
    if (b <= (1u << 20)) return (b + 255) & ~(size_t)255;
    size_t p2 = 1;
    while (p2 < b) p2 <<= 1;
    const size_t step = p2 >> 4;
    return (b + step - 1) / step * step;
}

// Caller holds g_pool_mu.  Frees every cached block (of one device, or of all when dev < 0).
size_t pool_release(int dev) {
    size_t freed = 0;
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (auto it = g_pool.begin(); it != g_pool.end();) {
        if (dev >= 0 && it->first.first != dev) { ++it; continue; }
        (void)hipSetDevice(it->first.first);
        (void)hipFree(it->second);
        freed += it->first.second;
        g_pool_bytes[it->first.first] -= it->first.second;
        it = g_pool.erase(it);
    }
    if (cur >= 0) (void)hipSetDevice(cur);
    return freed;
}

size_t pool_cap(int dev) {
    auto it = g_pool_cap.find(dev);
    if (it != g_pool_cap.end()) return it->second;
    size_t cap = 16ull << 30, total = 0;
    if (hipDeviceTotalMem(&total, dev) == hipSuccess && total) cap = total / 4 * 3;
    else (void)hipGetLastError();
    g_pool_cap[dev] = cap;
    return cap;
}
} // namespace

extern "C" uint64_t tt_trim_cache(void) {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    return pool_release(-1);
}

size_t dev_round(size_t bytes) { return round_size(bytes); }

size_t dev_bytes(const void *p) {
    if (!p) return 0;
    std::lock_guard<std::mutex> lock(g_pool_mu);
    auto it = g_live.find(const_cast<void *>(p));
    return it == g_live.end() ? 0 : it->second.size;
}

int dev_alloc(tt_graph *g, void **p, size_t bytes) {
    *p = nullptr;
    const size_t sz = round_size(bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(g_pool_mu);
    auto it = g_pool.find({dev, sz});
    if (it != g_pool.end()) {
        *p = it->second;
        g_pool.erase(it);
        g_pool_bytes[dev] -= sz;
    } else {
        hipError_t e = hipMalloc(p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            pool_release(dev);
            e = hipMalloc(p, sz);
        }
        if (e != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return fail(TT_E_NOMEM, "hipMalloc(" + std::to_string(sz) + " bytes) failed: " + hipGetErrorString(e));
        }
    }
    g_live[*p] = {sz, dev};
    if (g) g->bytes += sz;
    return TT_OK;
}

// Returns p to the cache; the caller guarantees no queued work still uses it.
void dev_free(tt_graph *g, void *p, size_t) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_pool_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    const Block blk = it->second;
    g_live.erase(it);
    if (g) g->bytes -= blk.size;
    if (g_pool_bytes[blk.device] + blk.size <= pool_cap(blk.device)) {
        g_pool.insert({{blk.device, blk.size}, p});
        g_pool_bytes[blk.device] += blk.size;
    } else {
        int cur = -1;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(blk.device);
        (void)hipFree(p);
        if (cur >= 0) (void)hipSetDevice(cur);
    }
}

int num_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    }
    return cus;
}

// ----------------------------------------------------------------------------- kernels
namespace {

constexpr uint32_t F_RANGE = 1, F_LOOP = 2, F_ZERO = 4, F_DUP = 8;

// Validation, the histogram of the weights by weight_bin (the graph's weight bins: the
// entries hold the same multiset of weights) and the graph's copy of the weights in input
// order.  Four edges per thread in flight; an LDS histogram per block, flushed with one global
// atomic per non-empty bin.
__global__ __launch_bounds__(256) void k_validate(const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                                                  uint64_t m, uint32_t n, uint32_t *flags,
                                                  unsigned long long *hist, uint32_t *w_copy) {
    __shared__ uint32_t h[WBINS];
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x) h[t] = 0;
    __syncthreads();
    uint32_t f = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < m; e0 += 4 * stride) {
        uint32_t a[4], b[4], x[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint64_t e = e0 + (uint64_t)i * stride;
            a[i] = b[i] = x[i] = 0;
            if (e < m) { a[i] = src[e]; b[i] = dst[e]; x[i] = w[e]; }
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
            if (e0 + (uint64_t)i * stride < m) {
                if (a[i] >= n || b[i] >= n) f |= F_RANGE;
                else if (a[i] == b[i]) f |= F_LOOP;
                if (x[i] == 0) f |= F_ZERO;
                atomicAdd(&h[weight_bin(x[i])], 1u);
                w_copy[e0 + (uint64_t)i * stride] = x[i];
            }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) f |= __shfl_xor(f, o, 64);
    if ((threadIdx.x & 63) == 0 && f) atomicOr(flags, f);
    __syncthreads();
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x)
        if (h[t]) atomicAdd(&hist[t], (unsigned long long)h[t]);
}

// Wave-level merging of atomics: in grid-stride loops the valid lanes are a prefix of the wave,
// and runs of equal keys in consecutive lanes (edge lists are often grouped by endpoint) are
// merged so that each run issues one atomic.  Returns the run's first lane for every lane.
struct WaveRuns {
    uint64_t heads;   // lanes that start a run
    int first;        // first lane of this lane's run
    int end;          // one past the last lane of this lane's run
};
__device__ __forceinline__ WaveRuns wave_runs(uint32_t key, bool valid) {
    const int lane = threadIdx.x & 63;
    const uint64_t vmask = __ballot(valid);
    const uint32_t pk = __shfl_up(key, 1, 64);
    const bool pv = lane > 0 && ((vmask >> (lane - 1)) & 1ull);
    const bool head = valid && (!pv || pk != key);
    WaveRuns r;
    r.heads = __ballot(head);
    const uint64_t upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const uint64_t before = r.heads & upto;
    r.first = before ? 63 - __builtin_clzll(before) : 0;
    const uint64_t after = lane == 63 ? 0ull : (r.heads >> (lane + 1)) << (lane + 1);
    const int nvalid = vmask ? 64 - __builtin_clzll(vmask) : 0;
    r.end = after ? __builtin_ctzll(after) : nvalid;
    return r;
}

__global__ __launch_bounds__(256) void k_degree(const uint32_t *src, const uint32_t *dst, uint64_t m, uint32_t *deg) {
    const int lane = threadIdx.x & 63;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < m; base += stride) {
        const uint64_t e = base + lane;
        const bool valid = e < m;
        const uint32_t a = valid ? src[e] : 0u, b = valid ? dst[e] : 0u;
        WaveRuns ra = wave_runs(a, valid);
        if (valid && ra.first == lane) atomicAdd(&deg[a], (uint32_t)(ra.end - lane));
        WaveRuns rb = wave_runs(b, valid);
        if (valid && rb.first == lane) atomicAdd(&deg[b], (uint32_t)(rb.end - lane));
    }
}

// tail of the oriented edge: the endpoint lower in (degree, ID) order
__device__ inline void orient(uint32_t a, uint32_t b, const uint32_t *deg, uint32_t &tail, uint32_t &head) {
    uint32_t da = deg[a], db = deg[b];
    bool a_low = da < db || (da == db && a < b);
    tail = a_low ? a : b;
    head = a_low ? b : a;
}

// Out-degree of every tail; each edge keeps its tail and its slot inside the tail's row (the
// value its atomic returned), so the scatter needs neither the degrees nor atomics.
__global__ __launch_bounds__(256) void k_outdeg(const uint32_t *src, const uint32_t *dst, uint64_t m,
                                                const uint32_t *deg, uint32_t *outdeg, uint32_t *etail,
                                                uint32_t *eslot) {
    const int lane = threadIdx.x & 63;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < m; base += stride) {
        const uint64_t e = base + lane;
        const bool valid = e < m;
        uint32_t t = 0, h = 0;
        if (valid) orient(src[e], dst[e], deg, t, h);
        WaveRuns r = wave_runs(t, valid);
        uint32_t slot = 0;
        if (valid && r.first == lane) slot = atomicAdd(&outdeg[t], (uint32_t)(r.end - lane));
        slot = __shfl(slot, r.first, 64) + (uint32_t)(lane - r.first);
        if (valid) {
            etail[e] = t;
            eslot[e] = slot;
        }
    }
}

// Scatters every edge into its tail's row (rows unsorted) as one 16-byte record.
__global__ __launch_bounds__(256) void k_scatter(const uint32_t *src, const uint32_t *dst, const uint32_t *w, uint64_t m,
                                                 const uint32_t *etail, const uint32_t *eslot, const uint64_t *rowp,
                                                 uint4 *rec) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        const uint32_t t = etail[e];
        const uint32_t h = src[e] ^ dst[e] ^ t; // the other endpoint
        rec[rowp[t] + eslot[e]] = make_uint4(h, w[e], (uint32_t)e, t); // (head, weight, edge, tail)
    }
}

// opos[eid[p]] = p: the entry position of every input edge (needed by edge sampling only).
__global__ __launch_bounds__(256) void k_make_opos(const uint32_t *eid, uint64_t m, uint32_t *opos) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += stride) opos[eid[p]] = (uint32_t)p;
}

// ----------------------------------------------------------------------------- partitioned front half
// Degrees, row lengths and the row-grouped records without global atomics on vertices:
// vertices are split into buckets of 2^rb consecutive IDs; a partition block takes a contiguous
// chunk of edges and its per-bucket counts form a bucket-major matrix M[b * nblk + blk] whose
// exclusive scan gives each (bucket, block) its range of a bucket-ordered array.  A bucket
// block then owns its vertices' counters in LDS.
constexpr uint32_t PART_MAX_BUCKETS = 8192; // LDS bins of a partition block
constexpr uint32_t PART_MAX_R = 16384;      // vertices per bucket (LDS counters of a bucket block)

struct PartGeom {
    uint32_t rb, nbk, nblk; // bucket shift, buckets, partition blocks
    uint64_t per;           // edges per partition block
};

// Partition blocks of 512 threads: their LDS (one counter per bucket) allows 4-5 blocks per
// CU, and the grid has at most 1,024 blocks, so the block size sets the waves in flight.
constexpr int PART_THREADS = 512;
// The scatter of the 16-byte records takes blocks twice as long, of twice the threads: half as
// many (bucket, block) ranges are written at once, so more of their partly written lines are
// combined before they leave the caches (49 -> 41 ms on the 2B-edge graph; the counting and
// endpoint passes are slower with the longer blocks, so they keep theirs).
constexpr int REC_THREADS = 1024;
// Bucket blocks (one per bucket, 64 KB of LDS per array of per-vertex counters) of 1,024 threads.
constexpr int BUCKET_THREADS = 1024;
// Items per thread and loop trip in the partition passes: their loads are issued together
// (one at a time, each trip waited on its load before the LDS atomic could start).
constexpr int PART_UNROLL = 4;

__global__ __launch_bounds__(PART_THREADS) void k_part_count_ends(const uint32_t *src, const uint32_t *dst, uint64_t m,
                                                         PartGeom G, uint32_t *M) {
    __shared__ uint32_t h[PART_MAX_BUCKETS];
    for (uint32_t b = threadIdx.x; b < G.nbk; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * G.per, hi = lo + G.per < m ? lo + G.per : m;
    for (uint64_t e0 = lo + threadIdx.x; e0 < hi; e0 += PART_UNROLL * blockDim.x) {
        uint32_t a[PART_UNROLL], d[PART_UNROLL];
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t e = e0 + (uint64_t)i * blockDim.x;
            if (e < hi) { a[i] = src[e]; d[i] = dst[e]; }
        }
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++)
            if (e0 + (uint64_t)i * blockDim.x < hi) {
                atomicAdd(&h[a[i] >> G.rb], 1u);
                atomicAdd(&h[d[i] >> G.rb], 1u);
            }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < G.nbk; b += blockDim.x) M[(uint64_t)b * G.nblk + blockIdx.x] = h[b];
}

// Both ends of every edge into bucket order.  C: the cursor type (32-bit when the output has
// fewer than 2^32 entries, which halves the block's LDS).
template <typename C>
__global__ __launch_bounds__(PART_THREADS) void k_part_ends(const uint32_t *src, const uint32_t *dst, uint64_t m,
                                                            PartGeom G, const uint64_t *off, uint32_t *ep) {
    __shared__ C cur[PART_MAX_BUCKETS];
    for (uint32_t b = threadIdx.x; b < G.nbk; b += blockDim.x) cur[b] = (C)off[(uint64_t)b * G.nblk + blockIdx.x];
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * G.per, hi = lo + G.per < m ? lo + G.per : m;
    for (uint64_t e0 = lo + threadIdx.x; e0 < hi; e0 += PART_UNROLL * blockDim.x) {
        uint32_t a[PART_UNROLL], d[PART_UNROLL];
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t e = e0 + (uint64_t)i * blockDim.x;
            if (e < hi) { a[i] = src[e]; d[i] = dst[e]; }
        }
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++)
            if (e0 + (uint64_t)i * blockDim.x < hi) {
                ep[atomicAdd(&cur[a[i] >> G.rb], (C)1)] = a[i];
                ep[atomicAdd(&cur[d[i] >> G.rb], (C)1)] = d[i];
            }
    }
}

// Degrees of bucket b's vertices from its endpoints ep[off(b, 0) .. off(b + 1, 0)).
__global__ __launch_bounds__(BUCKET_THREADS) void k_bucket_degree(const uint32_t *ep, const uint64_t *off, uint64_t total,
                                                       PartGeom G, uint32_t n, uint32_t *deg) {
    __shared__ uint32_t c[PART_MAX_R];
    const uint32_t b = blockIdx.x, R = 1u << G.rb;
    const uint64_t base = (uint64_t)b << G.rb;
    for (uint32_t i = threadIdx.x; i < R; i += blockDim.x) c[i] = 0;
    __syncthreads();
    const uint64_t lo = off[(uint64_t)b * G.nblk], hi = b + 1 < G.nbk ? off[(uint64_t)(b + 1) * G.nblk] : total;
    for (uint64_t j0 = lo + threadIdx.x; j0 < hi; j0 += PART_UNROLL * blockDim.x) {
        uint32_t x[PART_UNROLL];
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t j = j0 + (uint64_t)i * blockDim.x;
            if (j < hi) x[i] = ep[j];
        }
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++)
            if (j0 + (uint64_t)i * blockDim.x < hi) atomicAdd(&c[(uint32_t)(x[i] - base)], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < R; i += blockDim.x)
        if (base + i < n) deg[base + i] = c[i];
}

// The tail of every edge (kept in etail) and tails per (bucket, block).
__global__ __launch_bounds__(PART_THREADS) void k_part_count_tails(const uint32_t *src, const uint32_t *dst, uint64_t m,
                                                          PartGeom G, const uint32_t *deg, uint32_t *etail,
                                                          uint32_t *M) {
    __shared__ uint32_t h[PART_MAX_BUCKETS];
    for (uint32_t b = threadIdx.x; b < G.nbk; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * G.per, hi = lo + G.per < m ? lo + G.per : m;
    for (uint64_t e0 = lo + threadIdx.x; e0 < hi; e0 += PART_UNROLL * blockDim.x) {
        uint32_t a[PART_UNROLL], d[PART_UNROLL];
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t e = e0 + (uint64_t)i * blockDim.x;
            if (e < hi) { a[i] = src[e]; d[i] = dst[e]; }
        }
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t e = e0 + (uint64_t)i * blockDim.x;
            if (e < hi) {
                uint32_t t, hd;
                orient(a[i], d[i], deg, t, hd);
                etail[e] = t;
                atomicAdd(&h[t >> G.rb], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < G.nbk; b += blockDim.x) M[(uint64_t)b * G.nblk + blockIdx.x] = h[b];
}

// Counts per (bucket, record-scatter block) from those per (bucket, orientation block): scatter
// block k covers orientation blocks 2k and 2k + 1.
__global__ __launch_bounds__(256) void k_pair_blocks(const uint32_t *Mf, uint32_t nbk, uint32_t nf, uint32_t nc,
                                                     uint32_t *Mc) {
    const uint64_t total = (uint64_t)nbk * nc;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t b = i / nc;
        const uint32_t k = (uint32_t)(i - b * nc);
        const uint64_t f = b * nf + 2ull * k;
        Mc[i] = Mf[f] + (2 * k + 1 < nf ? Mf[f + 1] : 0u);
    }
}

// Every edge as a 16-byte record (head, weight, edge, tail) into tail-bucket order.
template <typename C>
__global__ __launch_bounds__(REC_THREADS) void k_part_edges(const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                                                             uint64_t m, PartGeom G, const uint32_t *etail,
                                                             const uint64_t *off, uint4 *part) {
    __shared__ C cur[PART_MAX_BUCKETS];
    for (uint32_t b = threadIdx.x; b < G.nbk; b += blockDim.x) cur[b] = (C)off[(uint64_t)b * G.nblk + blockIdx.x];
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * G.per, hi = lo + G.per < m ? lo + G.per : m;
    for (uint64_t e0 = lo + threadIdx.x; e0 < hi; e0 += PART_UNROLL * blockDim.x) {
        uint4 r[PART_UNROLL];
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t e = e0 + (uint64_t)i * blockDim.x;
            if (e < hi) {
                const uint32_t t = etail[e];
                r[i] = make_uint4(src[e] ^ dst[e] ^ t, w[e], (uint32_t)e, t);
            }
        }
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++)
            if (e0 + (uint64_t)i * blockDim.x < hi) part[atomicAdd(&cur[r[i].w >> G.rb], (C)1)] = r[i];
    }
}

// Second level of the endpoint grouping.  With many buckets a partition block keeps too many
// partly written lines open at once (one per bucket) for L2 to combine them, so the first level
// groups the endpoints by coarse buckets of 2^s2 buckets (cs = rb + s2) and this level refines
// each coarse group.  The input is grouped by coarse bucket, so a block's chunk [lo, hi)
// touches only the buckets of its first to last coarse bucket: a window [fb0, fb1) of at most
// nbk buckets.
struct SegGeom {
    uint32_t rb, cs, s2, nbk, nblk; // bucket shift, coarse shift, cs - rb, buckets, blocks
    uint64_t per;                   // endpoints per block
};

__device__ __forceinline__ bool seg_window(const uint32_t *in, uint64_t total, const SegGeom &G, uint64_t &lo,
                                           uint64_t &hi, uint32_t &fb0, uint32_t &fb1) {
    lo = (uint64_t)blockIdx.x * G.per;
    hi = lo + G.per < total ? lo + G.per : total;
    if (lo >= hi) return false;
    const uint32_t first = in[lo] >> G.cs, last = in[hi - 1] >> G.cs;
    fb0 = first << G.s2;
    const uint64_t e = (uint64_t)(last + 1) << G.s2;
    fb1 = e < G.nbk ? (uint32_t)e : G.nbk;
    return fb0 < fb1;
}

// Endpoints per (bucket, block); entries outside the block's window stay zero (cleared before).
__global__ __launch_bounds__(PART_THREADS) void k_seg_count(const uint32_t *in, uint64_t total, SegGeom G,
                                                            uint32_t *M) {
    __shared__ uint32_t h[PART_MAX_BUCKETS];
    uint64_t lo, hi;
    uint32_t fb0, fb1;
    if (!seg_window(in, total, G, lo, hi, fb0, fb1)) return;
    const uint32_t W = fb1 - fb0;
    for (uint32_t b = threadIdx.x; b < W; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (uint64_t e0 = lo + threadIdx.x; e0 < hi; e0 += PART_UNROLL * blockDim.x) {
        uint32_t x[PART_UNROLL];
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t e = e0 + (uint64_t)i * blockDim.x;
            if (e < hi) x[i] = in[e];
        }
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++)
            if (e0 + (uint64_t)i * blockDim.x < hi) {
                const uint32_t b = (x[i] >> G.rb) - fb0;
                if (b < W) atomicAdd(&h[b], 1u);
            }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < W; b += blockDim.x) M[(uint64_t)(fb0 + b) * G.nblk + blockIdx.x] = h[b];
}

// C: the cursor type, as in k_part_ends.
template <typename C>
__global__ __launch_bounds__(PART_THREADS) void k_seg_scatter(const uint32_t *in, uint64_t total, SegGeom G,
                                                              const uint64_t *off, uint32_t *out) {
    __shared__ C cur[PART_MAX_BUCKETS];
    uint64_t lo, hi;
    uint32_t fb0, fb1;
    if (!seg_window(in, total, G, lo, hi, fb0, fb1)) return;
    const uint32_t W = fb1 - fb0;
    for (uint32_t b = threadIdx.x; b < W; b += blockDim.x) cur[b] = (C)off[(uint64_t)(fb0 + b) * G.nblk + blockIdx.x];
    __syncthreads();
    for (uint64_t e0 = lo + threadIdx.x; e0 < hi; e0 += PART_UNROLL * blockDim.x) {
        uint32_t x[PART_UNROLL];
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t e = e0 + (uint64_t)i * blockDim.x;
            if (e < hi) x[i] = in[e];
        }
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++)
            if (e0 + (uint64_t)i * blockDim.x < hi) {
                const uint32_t b = (x[i] >> G.rb) - fb0;
                if (b < W) out[atomicAdd(&cur[b], (C)1)] = x[i];
            }
    }
}

// Rows of bucket b: records per tail (row lengths) and the largest weight per tail (row
// maxima), the lengths' exclusive scan from the bucket's first record (row starts, vertex
// order), then every record at its row's next slot.
__global__ __launch_bounds__(BUCKET_THREADS) void k_bucket_rows(const uint4 *part, const uint64_t *off, uint64_t m, PartGeom G,
                                                     uint32_t n, uint32_t *rlen, uint32_t *maxw, uint64_t *rowp,
                                                     uint4 *rec) {
    __shared__ uint32_t c[PART_MAX_R], mx[PART_MAX_R];
    __shared__ uint32_t wsum[BUCKET_THREADS / 64];
    const uint32_t b = blockIdx.x, R = 1u << G.rb, lane = threadIdx.x & 63, wib = threadIdx.x >> 6;
    const uint64_t base = (uint64_t)b << G.rb;
    for (uint32_t i = threadIdx.x; i < R; i += blockDim.x) c[i] = mx[i] = 0;
    __syncthreads();
    const uint64_t lo = off[(uint64_t)b * G.nblk], hi = b + 1 < G.nbk ? off[(uint64_t)(b + 1) * G.nblk] : m;
    for (uint64_t j0 = lo + threadIdx.x; j0 < hi; j0 += PART_UNROLL * blockDim.x) {
        uint2 x[PART_UNROLL]; // (tail, weight)
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t j = j0 + (uint64_t)i * blockDim.x;
            if (j < hi) {
                const uint4 r = part[j];
                x[i] = make_uint2(r.w, r.y);
            }
        }
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++)
            if (j0 + (uint64_t)i * blockDim.x < hi) {
                const uint32_t t = (uint32_t)(x[i].x - base);
                atomicAdd(&c[t], 1u);
                atomicMax(&mx[t], x[i].y);
            }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < R; i += blockDim.x)
        if (base + i < n) maxw[base + i] = mx[i];
    // thread t owns counters [t*per, t*per + per)
    const uint32_t per = (R + BUCKET_THREADS - 1) / BUCKET_THREADS;
    uint32_t sum = 0;
    for (uint32_t k = 0; k < per; k++) {
        const uint32_t i = threadIdx.x * per + k;
        if (i < R) {
            sum += c[i];
            if (base + i < n) rlen[base + i] = c[i];
        }
    }
    const uint32_t incl = wave_incl_scan(sum);
    if (lane == 63) wsum[wib] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (uint32_t w = 0; w < wib; w++) run += wsum[w];
    for (uint32_t k = 0; k < per; k++) {
        const uint32_t i = threadIdx.x * per + k;
        if (i < R) {
            const uint32_t x = c[i];
            c[i] = run;
            if (base + i < n) rowp[base + i] = lo + run;
            run += x;
        }
    }
    if (b == G.nbk - 1 && threadIdx.x == 0) rowp[n] = m;
    __syncthreads();
    for (uint64_t j0 = lo + threadIdx.x; j0 < hi; j0 += PART_UNROLL * blockDim.x) {
        uint4 r[PART_UNROLL];
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++) {
            const uint64_t j = j0 + (uint64_t)i * blockDim.x;
            if (j < hi) r[i] = part[j];
        }
#pragma unroll
        for (int i = 0; i < PART_UNROLL; i++)
            if (j0 + (uint64_t)i * blockDim.x < hi) rec[lo + atomicAdd(&c[(uint32_t)(r[i].w - base)], 1u)] = r[i];
    }
}

constexpr int BIG_TILE = 2048;

// One block per long row: bitonic sort of 2048-entry tiles in LDS, then stable merges by
// rank (each element finds its place in the sibling run by binary search).
template <typename K>
__global__ __launch_bounds__(256) void k_sort_big_rows(const uint64_t *rstart, const uint32_t *rlen, const uint32_t *big,
                                                       uint32_t nbig, K *key, uint32_t *p1, uint32_t *p2, K *tkey,
                                                       uint32_t *tp1, uint32_t *tp2) {
    __shared__ K sk[BIG_TILE];
    __shared__ uint32_t s1[BIG_TILE], s2[BIG_TILE];
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const uint32_t row = big[bi];
        const uint64_t b = rstart[row];
        const uint32_t len = rlen[row];
        for (uint32_t t0 = 0; t0 < len; t0 += BIG_TILE) {
            const uint32_t tl = min((uint32_t)BIG_TILE, len - t0);
            uint32_t P = 1;
            while (P < tl) P <<= 1;
            for (uint32_t t = threadIdx.x; t < P; t += blockDim.x) {
                if (t < tl) {
                    sk[t] = key[b + t0 + t];
                    s1[t] = p1[b + t0 + t];
                    s2[t] = p2 ? p2[b + t0 + t] : 0u;
                } else {
                    sk[t] = ~K(0); s1[t] = 0; s2[t] = 0;
                }
            }
            __syncthreads();
            for (uint32_t size = 2; size <= P; size <<= 1) {
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                        uint32_t i = 2 * t - (t & (stride - 1)), j = i + stride;
                        bool asc = (i & size) == 0;
                        if ((sk[i] > sk[j]) == asc) {
                            K kk = sk[i]; sk[i] = sk[j]; sk[j] = kk;
                            uint32_t x = s1[i]; s1[i] = s1[j]; s1[j] = x;
                            x = s2[i]; s2[i] = s2[j]; s2[j] = x;
                        }
                    }
                    __syncthreads();
                }
            }
            for (uint32_t t = threadIdx.x; t < tl; t += blockDim.x) {
                key[b + t0 + t] = sk[t];
                p1[b + t0 + t] = s1[t];
                if (p2) p2[b + t0 + t] = s2[t];
            }
            __syncthreads();
        }
        K *ik = key + b, *ok = tkey + b;
        uint32_t *i1 = p1 + b, *o1 = tp1 + b;
        uint32_t *i2 = p2 ? p2 + b : nullptr, *o2 = p2 ? tp2 + b : nullptr;
        bool in_tmp = false;
        for (uint32_t R = BIG_TILE; R < len; R <<= 1) {
            for (uint32_t x = threadIdx.x; x < len; x += blockDim.x) {
                const uint32_t r = x / R, i = x - r * R, base = (r & ~1u) * R;
                const K kx = ik[x];
                uint32_t lo, hi;
                const bool left = (r & 1u) == 0;
                if (left) { lo = (r + 1) * R; hi = min((r + 2) * R, len); if (lo > len) lo = len; }
                else { lo = (r - 1) * R; hi = r * R; }
                const uint32_t o0 = lo;
                while (lo < hi) { // lower_bound from the left run, upper_bound from the right run
                    uint32_t mid = (lo + hi) >> 1;
                    bool go = left ? (ik[mid] < kx) : (ik[mid] <= kx);
                    if (go) lo = mid + 1; else hi = mid;
                }
                const uint32_t pos = base + i + (lo - o0);
                ok[pos] = kx;
                o1[pos] = i1[x];
                if (i2) o2[pos] = i2[x];
            }
            __syncthreads();
            { K *t = ik; ik = ok; ok = t; }
            { uint32_t *t = i1; i1 = o1; o1 = t; }
            { uint32_t *t = i2; i2 = o2; o2 = t; }
            in_tmp = !in_tmp;
        }
        if (in_tmp) {
            for (uint32_t x = threadIdx.x; x < len; x += blockDim.x) {
                key[b + x] = ik[x];
                p1[b + x] = i1[x];
                if (p2) p2[b + x] = i2[x];
            }
        }
        __syncthreads();
    }
}

// Row maxima (maxw) and row bounds (hb = max(maxw[u], maxw[v] over out(u))) as streaming
// segmented reductions over the unsorted rows: each wave reduces the runs of equal tails in
// its 64 entries with shuffles and issues one atomicMax per run.
__device__ __forceinline__ uint32_t seg_max(uint32_t v, const WaveRuns &r) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_down(v, o, 64);
        if (lane + o < r.end) v = max(v, y);
    }
    return v;
}

__global__ __launch_bounds__(256) void k_row_max(const uint4 *rec, uint64_t m, uint32_t *maxw) {
    const int lane = threadIdx.x & 63;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < m; base += stride) {
        const uint64_t e = base + lane;
        const bool valid = e < m;
        const uint4 x = valid ? rec[e] : make_uint4(0u, 0u, 0u, 0u);
        const WaveRuns r = wave_runs(x.w, valid);
        const uint32_t v = seg_max(x.y, r);
        if (valid && r.first == lane) atomicMax(&maxw[x.w], v);
    }
}

// hb[u] = the largest row maximum among u's heads; hm0[j] (when kept) = the row maximum of
// record j's head, which the row ranking then places with the entry.
__global__ __launch_bounds__(256) void k_row_bound(const uint4 *rec, uint64_t m, const uint32_t *maxw, uint32_t *hb,
                                                   uint32_t *hm0) {
    const int lane = threadIdx.x & 63;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < m; base += stride) {
        const uint64_t e = base + lane;
        const bool valid = e < m;
        const uint4 x = valid ? rec[e] : make_uint4(0u, 0u, 0u, 0u);
        const WaveRuns r = wave_runs(x.w, valid);
        const uint32_t mh = valid ? maxw[x.x] : 0u;
        if (hm0 && valid) hm0[e] = mh;
        const uint32_t v = seg_max(mh, r);
        if (valid && r.first == lane) atomicMax(&hb[x.w], v);
    }
}

// Entries per weight_bin(hb[u]) (LDS-privatised histogram).
__global__ __launch_bounds__(256) void k_bin_entries(const uint32_t *hb, const uint32_t *rlen, uint32_t n,
                                                     unsigned long long *ecnt) {
    __shared__ unsigned long long h[WBINS];
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x) h[t] = 0;
    __syncthreads();
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (uint64_t)gridDim.x * blockDim.x)
        if (rlen[u]) atomicAdd(&h[weight_bin(hb[u])], (unsigned long long)rlen[u]);
    __syncthreads();
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x)
        if (h[t]) atomicAdd(&ecnt[t], h[t]);
}

constexpr int PLACE_ITEMS = 16;
// Graphs with at least this many vertices (row maxima of >= 64 MB) keep maxw of each entry's head.
constexpr uint32_t HMX_MIN_N = 1u << 24;

// Row starts grouped by bin: offsets inside the block come from LDS atomics, then one global
// atomic per (block, non-empty bin) reserves the block's range inside the bin.
__global__ __launch_bounds__(256) void k_place_rows(const uint32_t *hb, const uint32_t *rlen, uint32_t n,
                                                    const unsigned long long *binbase, unsigned long long *bincur,
                                                    uint64_t *rstart) {
    __shared__ unsigned long long lc[WBINS];
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x) lc[t] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * PLACE_ITEMS;
    unsigned long long off[PLACE_ITEMS];
#pragma unroll
    for (int it = 0; it < PLACE_ITEMS; it++) {
        const uint64_t u = base + (uint64_t)it * blockDim.x + threadIdx.x;
        off[it] = 0;
        if (u < n && rlen[u]) off[it] = atomicAdd(&lc[weight_bin(hb[u])], (unsigned long long)rlen[u]);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x)
        if (lc[t]) lc[t] = binbase[t] + atomicAdd(&bincur[t], lc[t]);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PLACE_ITEMS; it++) {
        const uint64_t u = base + (uint64_t)it * blockDim.x + threadIdx.x;
        if (u < n) rstart[u] = rlen[u] ? lc[weight_bin(hb[u])] + off[it] : 0;
    }
}

constexpr uint32_t SMALL_MAX = 64;   // rows ordered by a wave over a register window
constexpr uint32_t MID_MAX = 1024;   // rows ordered by a block in LDS
constexpr int RANK_ITEMS = 2;        // window of RANK_ITEMS * 64 entries per wave

// Writes one entry of a row (tail t, head c, weight w, input edge d) to both copies of the
// final layout: head order at rank r1, weight order at rank r2; records its tail and input edge.
__device__ __forceinline__ void put_entry(uint64_t P, uint32_t r1, uint32_t r2, uint32_t t, uint32_t c, uint32_t w,
                                          uint32_t d, uint32_t hm, uint32_t *col, uint32_t *wgt, uint32_t *eid,
                                          uint32_t *osrc, uint32_t *wcol, uint32_t *wwgt, uint32_t *wpos,
                                          uint32_t *hmx) {
    col[P + r1] = c;
    if (hmx) hmx[P + r1] = hm;
    wgt[P + r1] = w;
    eid[P + r1] = d;
    osrc[P + r1] = t;
    wcol[P + r2] = c;
    wwgt[P + r2] = w;
    wpos[P + r2] = (uint32_t)(P + r1);
}

// Ascending bitonic sort of 256*R 64-bit keys held by a block of 256 threads, thread t holding
// the keys at positions t + 256 r (r < R).  A compare-exchange at stride s pairs positions
// i and i ^ s: for s >= 256 both are in one thread (a register swap), for 64 <= s < 256 in
// two waves (an exchange through LDS), below 64 in one wave (a shuffle).
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int s) {
    const uint32_t lo = __shfl_xor((uint32_t)x, s, 64), hi = __shfl_xor((uint32_t)(x >> 32), s, 64);
    return ((uint64_t)hi << 32) | lo;
}

template <int R> __device__ __forceinline__ void block_bitonic(uint64_t (&k)[R], uint64_t *xch) {
    const uint32_t t = threadIdx.x;
    for (uint32_t size = 2; size <= 256u * R; size <<= 1) {
        for (uint32_t s = size >> 1; s > 0; s >>= 1) {
            if (s >= 256) {
                const uint32_t rs = s >> 8;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if (r & rs) continue;
                    const bool asc = ((t + 256u * r) & size) == 0;
                    const uint64_t x = k[r], y = k[r | rs];
                    if ((x > y) == asc) { k[r] = y; k[r | rs] = x; }
                }
                continue;
            }
            uint64_t other[R];
            if (s >= 64) {
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; r++) xch[t + 256u * r] = k[r];
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; r++) other[r] = xch[(t + 256u * r) ^ s];
            } else {
#pragma unroll
                for (int r = 0; r < R; r++) other[r] = shfl_xor_u64(k[r], (int)s);
            }
#pragma unroll
            for (int r = 0; r < R; r++) {
                const uint32_t i = t + 256u * r;
                const bool keep_min = ((i & s) == 0) == ((i & size) == 0);
                k[r] = keep_min ? min(k[r], other[r]) : max(k[r], other[r]);
            }
        }
    }
}

// Ascending bitonic sort of a wave's 64*R keys, lane l holding the keys at positions l + 64 r
// (r < R <= N): strides of 64 and more pair two registers of one lane, shorter ones two lanes.
template <int R, int N> __device__ __forceinline__ void wave_bitonic(uint64_t (&k)[N]) {
    static_assert(R <= N, "keys beyond the array");
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (uint32_t size = 2; size <= 64u * R; size <<= 1) {
#pragma unroll
        for (uint32_t s = size >> 1; s > 0; s >>= 1) {
            if (s >= 64) {
                const uint32_t rs = s >> 6;
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if (r & rs) continue;
                    const bool asc = ((lane + 64u * r) & size) == 0;
                    const uint64_t x = k[r], y = k[r | rs];
                    if ((x > y) == asc) { k[r] = y; k[r | rs] = x; }
                }
                continue;
            }
#pragma unroll
            for (int r = 0; r < R; r++) {
                const uint64_t o = shfl_xor_u64(k[r], (int)s);
                const uint32_t i = lane + 64u * r;
                const bool keep_min = ((i & s) == 0) == ((i & size) == 0);
                k[r] = keep_min ? min(k[r], o) : max(k[r], o);
            }
        }
    }
}

// Rows of at most SMALL_MAX entries.  Window w holds the rows that START in entries
// [64w, 64w+64) of the scatter layout; they end before 64w+128.  A wave stages that 128-entry
// window (heads and weights) in LDS and every lane counts its entries' ranks (by head ID; by
// weight desc, then head ID) over its own row only.  Equal heads in one row are a repeated pair.
__global__ __launch_bounds__(256) void k_rank_small(const uint4 *rec0, const uint64_t *rowp0, uint64_t m,
                                                    const uint64_t *rstart, const uint32_t *rlen, uint32_t *col,
                                                    uint32_t *wgt, uint32_t *eid, uint32_t *osrc,
                                                    uint32_t *wcol, uint32_t *wwgt, uint32_t *wpos, uint32_t *flags,
                                                    const uint32_t *hm0, uint32_t *hmx) {
    __shared__ uint32_t sc[4][RANK_ITEMS * 64], sw[4][RANK_ITEMS * 64];
    const int lane = threadIdx.x & 63, wib = threadIdx.x >> 6;
    const uint64_t nw = (m + 63) / 64;
    bool dup = false;
    // the whole block steps through windows together, so __syncthreads is uniform
    for (uint64_t blk = (uint64_t)blockIdx.x * 4; blk < nw; blk += (uint64_t)gridDim.x * 4) {
        const uint64_t w0 = blk + wib;
        const uint64_t base = w0 * 64;
        uint32_t c[RANK_ITEMS], wt[RANK_ITEMS], d[RANK_ITEMS], t[RANK_ITEMS], rb[RANK_ITEMS], len[RANK_ITEMS], hv[RANK_ITEMS];
        uint64_t P[RANK_ITEMS]; // final row start, loaded before the ranking so that it is not waited on after
        bool mine[RANK_ITEMS];
#pragma unroll
        for (int k = 0; k < RANK_ITEMS; k++) {
            const uint64_t e = base + (uint64_t)k * 64 + lane;
            uint4 r = make_uint4(0u, 0u, 0u, 0u);
            mine[k] = false;
            rb[k] = len[k] = hv[k] = 0;
            P[k] = 0;
            if (w0 < nw && e < m) {
                r = rec0[e];
                if (hm0) hv[k] = hm0[e];
                const uint64_t b = rowp0[r.w];
                len[k] = rlen[r.w];
                mine[k] = b >= base && b < base + 64 && len[k] <= SMALL_MAX;
                rb[k] = (uint32_t)(b - base); // window-relative row start (valid when mine)
                if (mine[k]) P[k] = rstart[r.w];
            }
            c[k] = r.x; wt[k] = r.y; d[k] = r.z; t[k] = r.w;
            sc[wib][k * 64 + lane] = r.x;
            sw[wib][k * 64 + lane] = r.y;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RANK_ITEMS; k++) {
            if (!mine[k]) continue;
            const uint32_t me = (uint32_t)(k * 64 + lane);
            uint32_t r1 = 0, r2 = 0;
            for (uint32_t f = rb[k]; f < rb[k] + len[k]; f++) {
                const uint32_t cf = sc[wib][f], wf = sw[wib][f];
                const bool before_id = cf < c[k] || (cf == c[k] && f < me);
                r1 += before_id;
                r2 += wf > wt[k] || (wf == wt[k] && before_id);
                dup |= cf == c[k] && f != me;
            }
            put_entry(P[k], r1, r2, t[k], c[k], wt[k], d[k], hv[k], col, wgt, eid, osrc, wcol, wwgt, wpos, hmx);
        }
        __syncthreads();
    }
    if (__ballot(dup) && lane == 0) atomicOr(flags, F_DUP);
}

// Lists the rows that need the LDS (mid) or the sorting (big) path.  Each block owns a
// contiguous range of vertices: it counts its mid and big rows, reserves its part of each list
// with one global atomic, then writes them (a per-wave atomic on two counters serialises).
__global__ __launch_bounds__(256) void k_list_long(const uint32_t *rlen, uint32_t n, uint32_t *mid, uint32_t *nmid,
                                                   uint32_t *big, uint32_t *nbig) {
    __shared__ uint32_t wm[4], wb[4], bm0, bb0;
    const uint32_t lane = threadIdx.x & 63, wib = threadIdx.x >> 6;
    const uint64_t per = ((uint64_t)n + gridDim.x - 1) / gridDim.x;
    const uint64_t lo = (uint64_t)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    uint32_t cm = 0, cb = 0;
    for (uint64_t u = lo + threadIdx.x; u < hi; u += blockDim.x) {
        const uint32_t l = rlen[u];
        cm += l > SMALL_MAX && l <= MID_MAX;
        cb += l > MID_MAX;
    }
    cm = wave_sum(cm);
    cb = wave_sum(cb);
    if (lane == 0) { wm[wib] = cm; wb[wib] = cb; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tm = wm[0] + wm[1] + wm[2] + wm[3], tb = wb[0] + wb[1] + wb[2] + wb[3];
        bm0 = tm ? atomicAdd(nmid, tm) : 0u;
        bb0 = tb ? atomicAdd(nbig, tb) : 0u;
    }
    __syncthreads();
    uint32_t run_m = bm0, run_b = bb0; // block-uniform
    const uint64_t below = (1ull << lane) - 1ull;
    for (uint64_t it = lo; it < hi; it += blockDim.x) {
        const uint64_t u = it + threadIdx.x;
        const uint32_t l = u < hi ? rlen[u] : 0u;
        const bool isb = l > MID_MAX, ism = l > SMALL_MAX && l <= MID_MAX;
        const uint64_t bb = __ballot(isb), bm = __ballot(ism);
        __syncthreads(); // the previous iteration has read wm/wb
        if (lane == 0) { wm[wib] = (uint32_t)__popcll(bm); wb[wib] = (uint32_t)__popcll(bb); }
        __syncthreads();
        uint32_t om = run_m, ob = run_b;
        for (uint32_t w = 0; w < wib; w++) { om += wm[w]; ob += wb[w]; }
        if (ism) mid[om + __popcll(bm & below)] = (uint32_t)u;
        if (isb) big[ob + __popcll(bb & below)] = (uint32_t)u;
        run_m += wm[0] + wm[1] + wm[2] + wm[3];
        run_b += wb[0] + wb[1] + wb[2] + wb[3];
    }
}

// Rows of SMALL_MAX+1 .. MID_MAX entries: one block per row.  The row is staged in LDS and
// sorted twice by the block: by (head, position) for the head-sorted layout, then by (weight
// descending, head-sorted position) for the weight-sorted copy; both are written coalesced.
// Equal neighbouring heads after the first sort are a repeated pair.
template <int R>
__device__ __forceinline__ void rank_mid_row(uint32_t u, uint64_t b, uint64_t P, uint32_t len, const uint4 *rec0,
                                             uint32_t *sc, uint32_t *sw, uint32_t *sd, uint32_t *hc, uint32_t *hw,
                                             uint64_t *xch, uint32_t *col, uint32_t *wgt, uint32_t *eid,
                                             uint32_t *osrc, uint32_t *wcol, uint32_t *wwgt,
                                             uint32_t *wpos, const uint32_t *hm0, uint32_t *hmx, bool &dup) {
    const uint32_t t = threadIdx.x;
    uint64_t k[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t i = t + 256u * r;
        k[r] = ~0ull;
        if (i < len) {
            const uint4 x = rec0[b + i];
            sc[i] = x.x;
            sw[i] = x.y;
            sd[i] = x.z;
            k[r] = ((uint64_t)x.x << 32) | i;
        }
    }
    block_bitonic<R>(k, xch);
    __syncthreads(); // sc/sw/sd complete
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t s = t + 256u * r;
        if (s < len) {
            const uint32_t i = (uint32_t)k[r], c = sc[i], w = sw[i], d = sd[i];
            col[P + s] = c;
            wgt[P + s] = w;
            eid[P + s] = d;
            osrc[P + s] = u;
            if (hmx) hmx[P + s] = hm0[b + i];
            hc[s] = c;
            hw[s] = w;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t s = t + 256u * r;
        dup |= s + 1 < len && hc[s + 1] == hc[s];
        k[r] = s < len ? (((uint64_t)~hw[s] << 32) | s) : ~0ull;
    }
    block_bitonic<R>(k, xch);
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t s = t + 256u * r;
        if (s < len) {
            const uint32_t h = (uint32_t)k[r];
            wcol[P + s] = hc[h];
            wwgt[P + s] = hw[h];
            wpos[P + s] = (uint32_t)(P + h);
        }
    }
    __syncthreads(); // LDS is reused by the block's next row
}

// Rows of SMALL_MAX+1 .. WAVE_MID_MAX entries, one per wave: the same two orders as
// rank_mid_row, sorted in registers (up to four keys per lane) with the row staged in the
// wave's quarter of the block's LDS arrays.  Every thread of the block calls it (`have` false
// where the wave has no such row), so that its barriers are uniform.
constexpr uint32_t WAVE_MID_MAX = 256;

__device__ __forceinline__ void rank_mid_wave(bool have, uint32_t u, uint64_t b, uint64_t P, uint32_t len,
                                              const uint4 *rec0, uint32_t *sc, uint32_t *sw, uint32_t *sd,
                                              uint32_t *hc, uint32_t *hw, uint32_t *col, uint32_t *wgt, uint32_t *eid,
                                              uint32_t *osrc, uint32_t *wcol, uint32_t *wwgt, uint32_t *wpos,
                                              const uint32_t *hm0, uint32_t *hmx, bool &dup) {
    const uint32_t lane = threadIdx.x & 63, q = (threadIdx.x >> 6) * WAVE_MID_MAX;
    uint64_t k[4];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const uint32_t i = lane + 64u * r;
        k[r] = ~0ull;
        if (have && i < len) {
            const uint4 x = rec0[b + i];
            sc[q + i] = x.x;
            sw[q + i] = x.y;
            sd[q + i] = x.z;
            k[r] = ((uint64_t)x.x << 32) | i;
        }
    }
    if (have) {
        if (len <= 128) wave_bitonic<2>(k);
        else wave_bitonic<4>(k);
    }
    __syncthreads(); // the wave's staged row is complete
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const uint32_t s = lane + 64u * r;
        if (have && s < len) {
            const uint32_t i = (uint32_t)k[r], c = sc[q + i], w = sw[q + i], d = sd[q + i];
            col[P + s] = c;
            wgt[P + s] = w;
            eid[P + s] = d;
            osrc[P + s] = u;
            if (hmx) hmx[P + s] = hm0[b + i];
            hc[q + s] = c;
            hw[q + s] = w;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const uint32_t s = lane + 64u * r;
        const bool in = have && s < len;
        dup |= in && s + 1 < len && hc[q + s + 1] == hc[q + s];
        k[r] = in ? (((uint64_t)~hw[q + s] << 32) | s) : ~0ull;
    }
    if (have) {
        if (len <= 128) wave_bitonic<2>(k);
        else wave_bitonic<4>(k);
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const uint32_t s = lane + 64u * r;
        if (have && s < len) {
            const uint32_t h = (uint32_t)k[r];
            wcol[P + s] = hc[q + h];
            wwgt[P + s] = hw[q + h];
            wpos[P + s] = (uint32_t)(P + h);
        }
    }
    __syncthreads(); // LDS is reused by the block's next rows
}

// A block takes the mid rows in groups of four: each row of at most WAVE_MID_MAX entries goes
// to one wave, then the group's longer rows are ranked by the whole block, one at a time.
__global__ __launch_bounds__(256) void k_rank_mid(const uint32_t *mid, uint32_t nmid, const uint4 *rec0,
                                                  const uint64_t *rowp0, const uint64_t *rstart, const uint32_t *rlen,
                                                  uint32_t *col, uint32_t *wgt, uint32_t *eid, uint32_t *osrc,
                                                  uint32_t *wcol, uint32_t *wwgt, uint32_t *wpos,
                                                  uint32_t *flags, const uint32_t *hm0, uint32_t *hmx) {
    static_assert(MID_MAX == 1024, "rows are sorted as up to 4 keys per thread");
    __shared__ uint32_t sc[MID_MAX], sw[MID_MAX], sd[MID_MAX], hc[MID_MAX], hw[MID_MAX];
    __shared__ uint64_t xch[MID_MAX];
    static_assert(4 * WAVE_MID_MAX <= MID_MAX, "a wave's rows fit its quarter of the arrays");
    bool dup = false;
    const uint32_t ngrp = (nmid + 3) / 4, wi = threadIdx.x >> 6;
    for (uint32_t g = blockIdx.x; g < ngrp; g += gridDim.x) {
        {
            const uint32_t bi = 4 * g + wi;
            uint32_t u = 0, len = 0;
            uint64_t b = 0, P = 0;
            if (bi < nmid) {
                u = mid[bi];
                len = rlen[u];
                b = rowp0[u];
                P = rstart[u];
            }
            rank_mid_wave(bi < nmid && len <= WAVE_MID_MAX, u, b, P, len, rec0, sc, sw, sd, hc, hw, col, wgt, eid,
                          osrc, wcol, wwgt, wpos, hm0, hmx, dup);
        }
        for (uint32_t j = 0; j < 4 && 4 * g + j < nmid; j++) { // block-uniform
            const uint32_t u = mid[4 * g + j], len = rlen[u];
            if (len <= WAVE_MID_MAX) continue;
            const uint64_t b = rowp0[u], P = rstart[u];
            if (len <= 512)
                rank_mid_row<2>(u, b, P, len, rec0, sc, sw, sd, hc, hw, xch, col, wgt, eid, osrc, wcol, wwgt, wpos, hm0, hmx, dup);
            else
                rank_mid_row<4>(u, b, P, len, rec0, sc, sw, sd, hc, hw, xch, col, wgt, eid, osrc, wcol, wwgt, wpos, hm0, hmx, dup);
        }
    }
    if (__ballot(dup) && (threadIdx.x & 63) == 0) atomicOr(flags, F_DUP);
}

// Longest rows: copied to the final layout here, sorted by k_sort_big_rows, then finished below.
__global__ __launch_bounds__(256) void k_move_big(const uint32_t *big, uint32_t nbig, const uint64_t *rowp0,
                                                  const uint64_t *rstart, const uint32_t *rlen, const uint4 *rec0,
                                                  uint32_t *col, uint32_t *wgt, uint32_t *eid, uint32_t *osrc) {
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const uint32_t u = big[bi];
        const uint64_t a = rowp0[u], b = rstart[u];
        for (uint32_t t = threadIdx.x; t < rlen[u]; t += blockDim.x) {
            const uint4 r = rec0[a + t];
            col[b + t] = r.x;
            wgt[b + t] = r.y;
            eid[b + t] = r.z;
            osrc[b + t] = u;
        }
    }
}

// After the head-ID sort of the long rows: the duplicate check and the keys of their
// weight-sorted copy.
__global__ __launch_bounds__(256) void k_post_big(const uint32_t *big, uint32_t nbig, const uint64_t *rstart,
                                                  const uint32_t *rlen, const uint32_t *col, const uint32_t *wgt,
                                                  uint64_t *wkey, uint32_t *wpos, uint32_t *flags,
                                                  const uint32_t *maxw, uint32_t *hmx) {
    bool dup = false;
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const uint32_t u = big[bi];
        const uint64_t b = rstart[u];
        for (uint32_t t = threadIdx.x; t < rlen[u]; t += blockDim.x) {
            const uint32_t c = col[b + t];
            if (t > 0 && col[b + t - 1] == c) dup = true;
            wkey[b + t] = ((uint64_t)(~wgt[b + t]) << 32) | c; // ascending = weight desc, then ID
            wpos[b + t] = (uint32_t)(b + t);
            if (hmx) hmx[b + t] = maxw[c];
        }
    }
    if (__ballot(dup) && (threadIdx.x & 63) == 0) atomicOr(flags, F_DUP);
}

__global__ __launch_bounds__(256) void k_split_big(const uint32_t *big, uint32_t nbig, const uint64_t *rstart,
                                                   const uint32_t *rlen, const uint64_t *wkey, uint32_t *wcol,
                                                   uint32_t *wwgt) {
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const uint32_t u = big[bi];
        const uint64_t b = rstart[u];
        for (uint32_t t = threadIdx.x; t < rlen[u]; t += blockDim.x) {
            const uint64_t k = wkey[b + t];
            wcol[b + t] = (uint32_t)k;
            wwgt[b + t] = ~(uint32_t)(k >> 32);
        }
    }
}

// Entries grouped by descending weight_bin(weight), for the bins in [blo, bhi): LDS offsets
// inside the block, one global atomic per (block, non-empty bin) to reserve the block's range
// inside the bin.
__global__ __launch_bounds__(256) void k_place_entries(const uint32_t *osrc, const uint32_t *col, const uint32_t *wgt,
                                                       uint64_t m, uint32_t blo, uint32_t bhi,
                                                       const unsigned long long *binbase,
                                                       unsigned long long *bincur, const uint32_t *hmx, uint32_t *ws_src,
                                                       uint32_t *ws_col, uint32_t *ws_wgt, uint32_t *ws_pos,
                                                       uint32_t *ws_hmx) {
    // counters only for the bins placed by this call, [blo, bhi): a call usually places a few
    // high bins, and clearing and scanning all 2,048 per block cost more than the block's items
    __shared__ uint32_t lc[WBINS];
    __shared__ unsigned long long lb[WBINS];
    const uint32_t nb = bhi - blo;
    for (uint32_t t = threadIdx.x; t < nb; t += blockDim.x) lc[t] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * PLACE_ITEMS;
    uint32_t off[PLACE_ITEMS], bin[PLACE_ITEMS], wv[PLACE_ITEMS]; // bin ~0u: not placed here
#pragma unroll
    for (int it = 0; it < PLACE_ITEMS; it++) {
        const uint64_t e = base + (uint64_t)it * blockDim.x + threadIdx.x;
        off[it] = 0;
        bin[it] = ~0u;
        wv[it] = 0;
        if (e < m) {
            wv[it] = wgt[e];
            const uint32_t b = weight_bin(wv[it]);
            if (b >= blo && b < bhi) {
                bin[it] = b - blo;
                off[it] = atomicAdd(&lc[b - blo], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < nb; t += blockDim.x)
        if (lc[t]) lb[t] = binbase[blo + t] + atomicAdd(&bincur[blo + t], (unsigned long long)lc[t]);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PLACE_ITEMS; it++) {
        const uint64_t e = base + (uint64_t)it * blockDim.x + threadIdx.x;
        const uint32_t w = wv[it];
        if (bin[it] != ~0u) {
            const uint64_t d = lb[bin[it]] + off[it];
            ws_src[d] = osrc[e];
            ws_col[d] = col[e];
            ws_wgt[d] = w;
            ws_pos[d] = (uint32_t)e;
            if (hmx) ws_hmx[d] = hmx[e];
        }
    }
}

// The same placement by rows, for calls that place some bins only: a row's entries of bins
// [blo, bhi) are a run of its weight-sorted copy (weights descend along it), and a row whose
// maximum is below bin blo has none, so only the rows that hold such entries are read (the
// entry-order placement reads every weight and, as the placed entries are spread over the
// whole layout, nearly every line of the other arrays).  Each thread takes PLACE_ROWS rows.
constexpr int PLACE_ROWS = 4;

__global__ __launch_bounds__(256) void k_place_row_runs(const uint64_t *rstart, const uint32_t *rlen,
                                                        const uint32_t *maxw, uint32_t n, const uint32_t *wcol,
                                                        const uint32_t *wwgt, const uint32_t *wpos, uint32_t blo,
                                                        uint32_t bhi, const unsigned long long *binbase,
                                                        unsigned long long *bincur, const uint32_t *hmx,
                                                        uint32_t *ws_src, uint32_t *ws_col, uint32_t *ws_wgt,
                                                        uint32_t *ws_pos, uint32_t *ws_hmx) {
    __shared__ uint32_t lc[WBINS];
    __shared__ unsigned long long lb[WBINS];
    const uint32_t nb = bhi - blo;
    for (uint32_t t = threadIdx.x; t < nb; t += blockDim.x) lc[t] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * PLACE_ROWS;
    uint64_t P[PLACE_ROWS];
    uint32_t j0[PLACE_ROWS], j1[PLACE_ROWS]; // the run [j0, j1) of the row's weight-sorted copy
#pragma unroll
    for (int it = 0; it < PLACE_ROWS; it++) {
        const uint64_t u = base + (uint64_t)it * blockDim.x + threadIdx.x;
        P[it] = 0;
        j0[it] = j1[it] = 0;
        if (u < n && weight_bin(maxw[u]) >= blo) {
            const uint64_t b = rstart[u];
            const uint32_t len = rlen[u];
            uint32_t j = 0, bj = 0;
            while (j < len && (bj = weight_bin(wwgt[b + j])) >= bhi) j++; // placed by earlier calls
            j0[it] = j;
            while (j < len && bj >= blo) {
                atomicAdd(&lc[bj - blo], 1u);
                if (++j < len) bj = weight_bin(wwgt[b + j]);
            }
            P[it] = b;
            j1[it] = j;
        }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < nb; t += blockDim.x)
        if (lc[t]) {
            lb[t] = binbase[blo + t] + atomicAdd(&bincur[blo + t], (unsigned long long)lc[t]);
            lc[t] = 0;
        }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PLACE_ROWS; it++) {
        const uint32_t u = (uint32_t)(base + (uint64_t)it * blockDim.x + threadIdx.x);
        for (uint32_t j = j0[it]; j < j1[it]; j++) {
            const uint64_t e = P[it] + j;
            const uint32_t w = wwgt[e], bi = weight_bin(w) - blo, h = wpos[e];
            const uint64_t d = lb[bi] + atomicAdd(&lc[bi], 1u);
            ws_src[d] = u;
            ws_col[d] = wcol[e];
            ws_wgt[d] = w;
            ws_pos[d] = h;
            if (hmx) ws_hmx[d] = hmx[h];
        }
    }
}

__global__ __launch_bounds__(256) void k_pack_cw(const uint32_t *col, const uint32_t *wgt, uint64_t m, uint2 *cw) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
        cw[e] = make_uint2(col[e], wgt[e]);
}

unsigned grid_for(uint64_t items, unsigned per_block = 256) {
    uint64_t b = (items + per_block - 1) / per_block;
    uint64_t cap = (uint64_t)num_cus() * 16;
    if (b > cap) b = cap;
    if (b == 0) b = 1;
    return (unsigned)b;
}
unsigned wave_grid(uint64_t rows) { // one wave per row, grid-stride
    uint64_t b = (rows + 3) / 4;
    uint64_t cap = (uint64_t)num_cus() * 16;
    if (b > cap) b = cap;
    return (unsigned)(b ? b : 1);
}

void release(tt_graph *g) {
    if (!g) return;
    void *ptrs[] = {g->rstart, g->rlen,   g->col,    g->wgt,  g->osrc,    g->eid,   g->opos,
                    g->wcol,   g->wwgt,   g->wpos,   g->maxw, g->hb,      g->deg,   g->emark,
                    g->ws_src, g->ws_col, g->ws_wgt, g->ws_pos, g->in_w,  g->irstart, g->itail,
                    g->vinfo,  g->cw,     g->hmx,    g->ws_hmx, g->ws_base, g->srstart, g->scol,
                    g->sw,     g->srowp};
    for (void *p : ptrs) dev_free(g, p, 0);
    for (auto &t : g->tables) {
        dev_free(g, t.prefix, 0);
        dev_free(g, t.guide, 0);
        dev_free(g, t.scan_tmp, 0);
    }
    for (auto &o : g->bord) {
        void *op[] = {o.src, o.col, o.wgt, o.pos};
        for (void *p : op) dev_free(g, p, 0);
        o = BoundOrder();
    }
    ctx_release(&g->q);
}

// Temporary device buffers of one build, freed on every exit path.
struct Scratch {
    hipStream_t stream = nullptr;
    std::vector<std::pair<void *, size_t>> bufs;
    int get(void **p, size_t bytes) {
        int rc = dev_alloc(nullptr, p, bytes);
        if (!rc) bufs.push_back({*p, bytes});
        return rc;
    }
    void drop(void *p) {
        for (auto &b : bufs)
            if (b.first == p) { dev_free(nullptr, b.first, b.second); b.first = nullptr; }
    }
    ~Scratch() {
        if (stream) (void)hipStreamSynchronize(stream); // nothing queued may still use them
        for (auto &b : bufs)
            if (b.first) dev_free(nullptr, b.first, b.second);
    }
};

// Sorts the listed long rows by key K (ascending), carrying up to two u32 payloads, on stream s.
template <typename K>
int sort_big(tt_graph *g, Scratch &S, hipStream_t s, const uint64_t *rstart, const uint32_t *rlen, const uint32_t *big,
             uint32_t nbig, K *key, uint32_t *p1, uint32_t *p2) {
    if (!nbig) return TT_OK;
    const uint64_t m = g->m;
    K *tk = nullptr;
    uint32_t *t12 = nullptr;
    int rc;
    if ((rc = S.get((void **)&tk, (m + 1) * sizeof(K))) || (rc = S.get((void **)&t12, 2 * (m + 1) * 4))) return rc;
    const unsigned grid = nbig < 4096u ? nbig : 4096u;
    k_sort_big_rows<K><<<grid, 256, 0, s>>>(rstart, rlen, big, nbig, key, p1, p2, tk, t12, t12 + (m + 1));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    S.drop(tk);
    S.drop(t12);
    return TT_OK;
}

// Two more streams (default priority), for the ranking of the mid and of the long rows beside
// that of the small rows: the three classes write disjoint rows.  The streams are made once per
// device and kept for the process (making them for every build cost ~0.1 ms); builds that run
// at once share them, which orders their work but keeps each build's own order.  Both wait
// for what the build's stream has queued, and join() makes it wait for them; the destructor
// waits for them too, so that no scratch they use is freed under them (declare it after the
// Scratch).
static int device_side_streams(hipStream_t &a, hipStream_t &b) {
    static std::mutex mu;
    static std::map<int, std::pair<hipStream_t, hipStream_t>> made;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = made.find(dev);
    if (it == made.end()) {
        hipStream_t x = nullptr, y = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        if (hipStreamCreateWithFlags(&y, hipStreamNonBlocking) != hipSuccess) {
            (void)hipStreamDestroy(x);
            return fail(TT_E_DEVICE, "hipStreamCreateWithFlags failed");
        }
        it = made.emplace(dev, std::make_pair(x, y)).first;
    }
    a = it->second.first;
    b = it->second.second;
    return TT_OK;
}

struct SideStreams {
    hipStream_t mid = nullptr, big = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    int open(hipStream_t s) {
        int rc;
        if ((rc = device_side_streams(mid, big))) return rc;
        for (hipEvent_t &e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev[0], s));
        HIP_TRY(hipStreamWaitEvent(mid, ev[0], 0));
        HIP_TRY(hipStreamWaitEvent(big, ev[0], 0));
        return TT_OK;
    }
    int join(hipStream_t s) {
        HIP_TRY(hipEventRecord(ev[1], mid));
        HIP_TRY(hipEventRecord(ev[2], big));
        HIP_TRY(hipStreamWaitEvent(s, ev[1], 0));
        HIP_TRY(hipStreamWaitEvent(s, ev[2], 0));
        return TT_OK;
    }
    ~SideStreams() {
        for (hipStream_t x : {mid, big})
            if (x) (void)hipStreamSynchronize(x);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};
// Graphs with at least this many edges rank the three row classes concurrently (below it the
// streams' set-up is not repaid).
constexpr uint64_t SIDE_STREAMS_MIN_M = 1ull << 22;

// In-degrees of the oriented CSR (heads of all entries), runs merged per wave.
__global__ __launch_bounds__(256) void k_indeg(const uint32_t *col, uint64_t m, uint32_t *indeg) {
    const int lane = threadIdx.x & 63;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < m; base += stride) {
        const uint64_t e = base + lane;
        const bool valid = e < m;
        const uint32_t v = valid ? col[e] : 0u;
        const WaveRuns r = wave_runs(v, valid);
        if (valid && r.first == lane) atomicAdd(&indeg[v], (uint32_t)(r.end - lane));
    }
}

__global__ __launch_bounds__(256) void k_in_scatter(const uint32_t *col, const uint32_t *osrc, uint64_t m,
                                                    const uint64_t *irstart, uint32_t *cursor, uint32_t *itail) {
    const int lane = threadIdx.x & 63;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < m; base += stride) {
        const uint64_t e = base + lane;
        const bool valid = e < m;
        const uint32_t v = valid ? col[e] : 0u;
        const WaveRuns r = wave_runs(v, valid);
        uint32_t slot = 0;
        if (valid && r.first == lane) slot = atomicAdd(&cursor[v], (uint32_t)(r.end - lane));
        slot = __shfl(slot, r.first, 64) + (uint32_t)(lane - r.first);
        if (valid) itail[irstart[v] + slot] = osrc[e];
    }
}

// The intersection's per-vertex reads in one 16-byte record, and rows as (col, wgt) pairs.
__global__ __launch_bounds__(256) void k_pack_vinfo(const uint64_t *rstart, const uint32_t *rlen, const uint32_t *maxw,
                                                    uint64_t nn, VInfo *vi) {
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += (uint64_t)gridDim.x * blockDim.x)
        vi[v] = VInfo{rstart[v], rlen[v], maxw[v]};
}


} // namespace

// ----------------------------------------------------------------------------- build
// Buckets of 2^rb vertices, rb in [6, 14], at least ~2,048 buckets where n allows (bucket
// blocks fill the device); partition blocks of >= 8,192 edges, at most 1,024 of them (fewer,
// larger blocks measured slower for the counting and endpoint passes; the record scatter takes
// them in pairs, see REC_THREADS).
PartGeom part_geometry(uint32_t n, uint64_t m) {
    PartGeom G;
    uint32_t rb = 6;
    while (rb < 14 && ((uint64_t)n >> (rb + 1)) >= 2048) rb++;
    G.rb = rb;
    G.nbk = (uint32_t)(((uint64_t)n + (1ull << rb) - 1) >> rb);
    if (G.nbk == 0) G.nbk = 1;
    uint64_t nblk = (m + 8191) / 8192;
    if (nblk > 1024) nblk = 1024;
    if (nblk == 0) nblk = 1;
    G.per = (m + nblk - 1) / nblk;
    if (G.per == 0) G.per = 1;                    // m == 0
    G.nblk = (uint32_t)((m + G.per - 1) / G.per); // no empty trailing block
    if (G.nblk == 0) G.nblk = 1;
    return G;
}

// Blocks of the second partition level over `total` items (same block sizing as the first).
SegGeom seg_geometry(const PartGeom &P, uint32_t s2, uint64_t total) {
    SegGeom G;
    G.rb = P.rb;
    G.s2 = s2;
    G.cs = P.rb + s2;
    G.nbk = P.nbk;
    uint64_t nblk = (total + 8191) / 8192;
    if (nblk > 1024) nblk = 1024;
    if (nblk == 0) nblk = 1;
    G.per = (total + nblk - 1) / nblk;
    if (G.per == 0) G.per = 1;
    G.nblk = (uint32_t)((total + G.per - 1) / G.per);
    if (G.nblk == 0) G.nblk = 1;
    return G;
}

constexpr uint32_t PART_COARSE = 128; // at most this many buckets open per block and level

static int build_csr(tt_graph *g, const uint32_t *src, const uint32_t *dst, const uint32_t *w) {
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    hipStream_t s = g->stream;
    int rc;
    Scratch S;
    S.stream = s;
    uint32_t *flags = nullptr;
    unsigned long long *hist = nullptr; // entries per weight_bin, made by the validation pass
    if ((rc = S.get((void **)&flags, 16)) || (rc = S.get((void **)&hist, WBINS * 8)) ||
        (rc = dev_alloc(g, (void **)&g->in_w, (m + 1) * 4)))
        return rc;
    HIP_TRY(hipMemsetAsync(flags, 0, 16, s));
    HIP_TRY(hipMemsetAsync(hist, 0, WBINS * 8, s));
    if (m)
        k_validate<<<std::min<unsigned>(grid_for(m), (unsigned)num_cus() * 4), 256, 0, s>>>(src, dst, w, m, n, flags,
                                                                                            hist, g->in_w);
    uint32_t hf[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf[0] & F_RANGE) return fail(TT_E_VERTEX_RANGE, "an edge endpoint is >= n");
    if (hf[0] & F_LOOP) return fail(TT_E_SELF_LOOP, "the graph has a self-loop");
    if (hf[0] & F_ZERO) return fail(TT_E_ZERO_WEIGHT, "an edge weight is 0");

    const uint64_t nn = (uint64_t)n + 1;
    uint64_t *rowp0 = nullptr;
    uint4 *rec0 = nullptr;
    uint32_t *big = nullptr, *mid = nullptr;
    if ((rc = dev_alloc(g, (void **)&g->deg, nn * 4)) || (rc = dev_alloc(g, (void **)&g->rstart, nn * 8)) ||
        (rc = dev_alloc(g, (void **)&g->rlen, nn * 4)) || (rc = dev_alloc(g, (void **)&g->maxw, nn * 4)) ||
        (rc = dev_alloc(g, (void **)&g->hb, nn * 4)) || (rc = dev_alloc(g, (void **)&g->col, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->wgt, (m + 1) * 4)) || (rc = dev_alloc(g, (void **)&g->osrc, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->eid, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->wcol, (m + 1) * 4)) || (rc = dev_alloc(g, (void **)&g->wwgt, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->wpos, (m + 1) * 4)) ||
        (rc = S.get((void **)&big, nn * 4)) ||
        (rc = S.get((void **)&mid, nn * 4)) || (rc = S.get((void **)&rowp0, (nn + 1) * 8)) ||
        (rc = S.get((void **)&rec0, (m + 1) * 16)))
        return rc;
    HIP_TRY(hipMemsetAsync(g->deg, 0, nn * 4, s));
    HIP_TRY(hipMemsetAsync(g->rlen, 0, nn * 4, s));
    HIP_TRY(hipMemsetAsync(g->maxw, 0, nn * 4, s));
    // rows in vertex order first (unsorted), rowp0[n] = m
    const PartGeom PG = part_geometry(n, m);
    if (m && PG.nbk <= PART_MAX_BUCKETS && (1u << PG.rb) <= PART_MAX_R) {
        // partitioned: endpoints and then records grouped by vertex bucket, counted in LDS.  With
        // more than PART_COARSE buckets the endpoints are grouped in two levels: coarse buckets
        // of 2^s2 buckets, then each coarse group refined (k_seg_count / k_seg_scatter).
        uint32_t s2 = 0;
        while ((PG.nbk >> s2) > PART_COARSE) s2++;
        PartGeom P1 = PG; // first level of the endpoint grouping: coarse buckets
        P1.rb = PG.rb + s2;
        P1.nbk = (uint32_t)(((uint64_t)n + (1ull << P1.rb) - 1) >> P1.rb);
        const SegGeom E2 = seg_geometry(PG, s2, 2 * m);
        PartGeom PE = PG; // bucket geometry of the final grouping of the endpoints
        if (s2) {
            PE.nblk = E2.nblk;
            PE.per = E2.per;
        }
        const uint64_t nm = std::max(std::max((uint64_t)P1.nbk * P1.nblk, (uint64_t)PE.nbk * PE.nblk),
                                     (uint64_t)PG.nbk * PG.nblk);
        uint32_t *M = nullptr;
        uint64_t *off = nullptr;
        void *scan_tmp = nullptr, *grouped = nullptr; // grouped: endpoints (8m B), then records (16m B)
        if ((rc = S.get((void **)&M, nm * 4)) || (rc = S.get((void **)&off, nm * 8)) ||
            (rc = S.get(&scan_tmp, scan_tmp_bytes(nm))) || (rc = S.get(&grouped, m * 16)))
            return rc;
        // first level into rec0 when a second follows (rec0 is written only by k_bucket_rows)
        uint32_t *ep1 = s2 ? (uint32_t *)rec0 : (uint32_t *)grouped;
        const bool ends32 = 2 * m < (1ull << 32);
        k_part_count_ends<<<P1.nblk, PART_THREADS, 0, s>>>(src, dst, m, P1, M);
        if ((rc = exclusive_scan_u32_to_u64(M, off, (uint64_t)P1.nbk * P1.nblk, s, nullptr, scan_tmp))) return rc;
        if (ends32) k_part_ends<uint32_t><<<P1.nblk, PART_THREADS, 0, s>>>(src, dst, m, P1, off, ep1);
        else k_part_ends<unsigned long long><<<P1.nblk, PART_THREADS, 0, s>>>(src, dst, m, P1, off, ep1);
        if (s2) {
            const uint64_t nme = (uint64_t)PE.nbk * PE.nblk;
            HIP_TRY(hipMemsetAsync(M, 0, nme * 4, s));
            k_seg_count<<<E2.nblk, PART_THREADS, 0, s>>>(ep1, 2 * m, E2, M);
            if ((rc = exclusive_scan_u32_to_u64(M, off, nme, s, nullptr, scan_tmp))) return rc;
            if (ends32) k_seg_scatter<uint32_t><<<E2.nblk, PART_THREADS, 0, s>>>(ep1, 2 * m, E2, off, (uint32_t *)grouped);
            else k_seg_scatter<unsigned long long><<<E2.nblk, PART_THREADS, 0, s>>>(ep1, 2 * m, E2, off, (uint32_t *)grouped);
        }
        k_bucket_degree<<<PE.nbk, BUCKET_THREADS, 0, s>>>((const uint32_t *)grouped, off, 2 * m, PE, n, g->deg);
        // records in one level (a second level measured no faster for the 16-byte records).
        // The weight-sorted head array holds each edge's tail until the row ranking fills it.
        // The scatter's blocks (PR) are pairs of the orientation pass's (PG).
        PartGeom PR = PG;
        PR.per = 2 * PG.per;
        PR.nblk = (uint32_t)((m + PR.per - 1) / PR.per);
        uint32_t *Mr = nullptr;
        if ((rc = S.get((void **)&Mr, (uint64_t)PR.nbk * PR.nblk * 4))) return rc;
        k_part_count_tails<<<PG.nblk, PART_THREADS, 0, s>>>(src, dst, m, PG, g->deg, g->wcol, M);
        k_pair_blocks<<<grid_for((uint64_t)PR.nbk * PR.nblk), 256, 0, s>>>(M, PG.nbk, PG.nblk, PR.nblk, Mr);
        if ((rc = exclusive_scan_u32_to_u64(Mr, off, (uint64_t)PR.nbk * PR.nblk, s, nullptr, scan_tmp))) return rc;
        if (m < (1ull << 32)) k_part_edges<uint32_t><<<PR.nblk, REC_THREADS, 0, s>>>(src, dst, w, m, PR, g->wcol, off, (uint4 *)grouped);
        else k_part_edges<unsigned long long><<<PR.nblk, REC_THREADS, 0, s>>>(src, dst, w, m, PR, g->wcol, off, (uint4 *)grouped);
        k_bucket_rows<<<PR.nbk, BUCKET_THREADS, 0, s>>>((const uint4 *)grouped, off, m, PR, n, g->rlen, g->maxw, rowp0,
                                                         rec0);
        HIP_TRY(hipGetLastError());
    } else {
        if (m) {
            k_degree<<<grid_for(m), 256, 0, s>>>(src, dst, m, g->deg);
            // the weight-sorted arrays are filled by the row ranking; until then they hold each
            // edge's tail and slot
            k_outdeg<<<grid_for(m), 256, 0, s>>>(src, dst, m, g->deg, g->rlen, g->wcol, g->wwgt);
        }
        void *scan_tmp = nullptr;
        if ((rc = S.get(&scan_tmp, scan_tmp_bytes(nn))) ||
            (rc = exclusive_scan_u32_to_u64(g->rlen, rowp0, nn, s, nullptr, scan_tmp)))
            return rc;
        if (m) k_scatter<<<grid_for(m), 256, 0, s>>>(src, dst, w, m, g->wcol, g->wwgt, rowp0, rec0);
        if (m) k_row_max<<<grid_for(m), 256, 0, s>>>(rec0, m, g->maxw); // (the bucket pass makes them above)
    }
    HIP_TRY(hipMemcpyAsync(g->hb, g->maxw, nn * 4, hipMemcpyDeviceToDevice, s));
    // The per-entry head maxima pay only where the row maxima no longer stay in the caches
    // (then the filter's gather of maxw[v] misses to HBM for nearly every streamed entry).  They
    // are gathered once, in record order, and placed by the row ranking with their entries.
    uint32_t *hm0 = nullptr;
    if (n >= HMX_MIN_N &&
        ((rc = dev_alloc(g, (void **)&g->hmx, (m + 1) * 4)) || (rc = S.get((void **)&hm0, (m + 1) * 4))))
        return rc;
    if (m) k_row_bound<<<grid_for(m), 256, 0, s>>>(rec0, m, g->maxw, g->hb, hm0);
    // layout by descending weight_bin(hb)
    unsigned long long *ecnt = nullptr, *bincur = nullptr, *binbase = nullptr;
    if ((rc = S.get((void **)&ecnt, WBINS * 8)) || (rc = S.get((void **)&bincur, WBINS * 8)) ||
        (rc = S.get((void **)&binbase, WBINS * 8)))
        return rc;
    HIP_TRY(hipMemsetAsync(ecnt, 0, WBINS * 8, s));
    HIP_TRY(hipMemsetAsync(bincur, 0, WBINS * 8, s));
    // (histograms: a few blocks per CU, so that each bin's global counter takes few atomics)
    if (n) k_bin_entries<<<std::min<unsigned>(grid_for(n), (unsigned)num_cus() * 4), 256, 0, s>>>(g->hb, g->rlen, n, ecnt);
    g->ebin.assign(WBINS, 0);
    g->ebase.assign(WBINS, 0);
    HIP_TRY(hipMemcpyAsync(g->ebin.data(), ecnt, WBINS * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    {
        uint64_t run = 0;
        for (int b = WBINS - 1; b >= 0; b--) { g->ebase[b] = run; run += g->ebin[b]; }
    }
    HIP_TRY(hipMemcpyAsync(binbase, g->ebase.data(), WBINS * 8, hipMemcpyHostToDevice, s));
    if (n) {
        const uint64_t per = 256ull * PLACE_ITEMS;
        k_place_rows<<<(unsigned)(((uint64_t)n + per - 1) / per), 256, 0, s>>>(g->hb, g->rlen, n, binbase, bincur, g->rstart);
    }
    // both row orders: counted ranks for rows up to SMALL_MAX entries, LDS sorts up to MID_MAX,
    // sorts in memory for longer ones; the three classes on three streams on large graphs
    HIP_TRY(hipMemsetAsync(flags + 1, 0, 8, s));
    if (n) k_list_long<<<grid_for(n, 4096), 256, 0, s>>>(g->rlen, n, mid, flags + 2, big, flags + 1);
    HIP_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint32_t nbig = hf[1], nmid = hf[2];
    SideStreams side;
    hipStream_t s_mid = s, s_big = s;
    if (m >= SIDE_STREAMS_MIN_M && (nmid || nbig)) {
        if ((rc = side.open(s))) return rc;
        s_mid = side.mid;
        s_big = side.big;
    }
    if (m) k_rank_small<<<grid_for(m), 256, 0, s>>>(rec0, rowp0, m, g->rstart, g->rlen, g->col, g->wgt, g->eid, g->osrc,
                                                    g->wcol, g->wwgt, g->wpos, flags, hm0, g->hmx);
    if (nmid) {
        const uint32_t ngrp = (nmid + 3) / 4; // groups of four rows
        const unsigned gm = ngrp < 8192u ? ngrp : 8192u;
        k_rank_mid<<<gm, 256, 0, s_mid>>>(mid, nmid, rec0, rowp0, g->rstart, g->rlen, g->col, g->wgt, g->eid, g->osrc,
                                          g->wcol, g->wwgt, g->wpos, flags, hm0, g->hmx);
    }
    if (nbig) {
        const unsigned gb = nbig < 4096u ? nbig : 4096u;
        k_move_big<<<gb, 256, 0, s_big>>>(big, nbig, rowp0, g->rstart, g->rlen, rec0, g->col, g->wgt, g->eid, g->osrc);
        if ((rc = sort_big<uint32_t>(g, S, s_big, g->rstart, g->rlen, big, nbig, g->col, g->wgt, g->eid))) return rc;
        uint64_t *wkey = nullptr;
        if ((rc = S.get((void **)&wkey, (m + 1) * 8))) return rc;
        k_post_big<<<gb, 256, 0, s_big>>>(big, nbig, g->rstart, g->rlen, g->col, g->wgt, wkey, g->wpos, flags, g->maxw,
                                          g->hmx);
        if ((rc = sort_big<uint64_t>(g, S, s_big, g->rstart, g->rlen, big, nbig, wkey, g->wpos, nullptr))) return rc;
        k_split_big<<<gb, 256, 0, s_big>>>(big, nbig, g->rstart, g->rlen, wkey, g->wcol, g->wwgt);
        HIP_TRY(hipStreamSynchronize(s_big)); // wkey is dropped below
        S.drop(wkey);
    }
    if (side.mid && (rc = side.join(s))) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    S.drop(rec0);
    g->whist.assign(WBINS, 0);
    HIP_TRY(hipMemcpyAsync(g->whist.data(), hist, WBINS * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    if (hf[0] & F_DUP) return fail(TT_E_DUP_EDGE, "the same unordered vertex pair appears twice");
    // an upper bound of the largest weight: the top of the highest non-empty bin
    g->wmax = 0;
    for (int b = WBINS - 1; b >= 0; b--)
        if (g->whist[b]) {
            // first weight of bin b+1, in 64 bits (it is 2^32 for the top bin)
            const uint32_t nb = (uint32_t)b + 1;
            const uint64_t up = nb < 64 ? nb : ((uint64_t)((nb - 64) % 64 + 64) << ((nb - 64) / 64));
            g->wmax = (uint32_t)std::min<uint64_t>(up - 1, 0xFFFFFFFFull);
            break;
        }
    // the weight-ordered stream of entries
    g->wbase.assign(WBINS, 0);
    {
        uint64_t run = 0;
        for (int b = WBINS - 1; b >= 0; b--) { g->wbase[b] = run; run += g->whist[b]; }
    }
    // (the stream itself is placed by the first query that streams it: ensure_weight_stream)
    // the (head, weight) pairs are packed after the ranking, once its scratch is returned (made
    // inside the ranking, their 16 GB on the 2B-edge graph raised the build's peak and the
    // allocator then had to return cached blocks to the driver in later queries)
    if ((rc = dev_alloc(g, (void **)&g->vinfo, nn * sizeof(VInfo))) || (rc = dev_alloc(g, (void **)&g->cw, (m + 1) * 8)))
        return rc;
    k_pack_vinfo<<<grid_for(nn), 256, 0, s>>>(g->rstart, g->rlen, g->maxw, nn, g->vinfo);
    if (m) k_pack_cw<<<grid_for(m), 256, 0, s>>>(g->col, g->wgt, m, g->cw);
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    return TT_OK;
}

// The entry position of every input edge (built once, on the first sampling query).
int ensure_opos(tt_graph *g, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g->init_mu);
    if (g->opos) return TT_OK;
    uint32_t *opos = nullptr;
    int rc = dev_alloc(g, (void **)&opos, (g->m + 1) * 4);
    if (rc) return rc;
    if (g->m) k_make_opos<<<grid_for(g->m), 256, 0, s>>>(g->eid, g->m, opos);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s)); // complete before other streams may see it
    g->opos = opos;
    return TT_OK;
}

// The entries in order of descending weight bin, placed down to bin `bin` at least (bins are
// placed on demand, as a query's band first needs them; on graphs of more than ws_all_at_once()
// entries each call places the bins from the requested one up to those already placed,
// extended down until the placed prefix holds WS_GROW times the requested one and at least
// m / WS_MIN_FRAC entries, so that a descending sequence of bands costs a few calls).  Each
// call writes only the new bins; it reads every row maximum and the rows that hold new bins.
constexpr uint64_t WS_GROW = 4, WS_MIN_FRAC = 1024;
// Up to this many entries one call places every bin: a call costs about a pass over all the
// weights whatever it writes (the 20M-entry graph: 0.22 ms for a partial placement, 0.37 ms for
// all of it), while on larger graphs the writes dominate (2B entries: all bins ~54 ms).  The
// environment variable TT_WS_ALL_AT_ONCE overrides it (tests use it to take the partial path on
// small graphs).
uint64_t ws_all_at_once() {
    const char *e = std::getenv("TT_WS_ALL_AT_ONCE");
    return e ? std::strtoull(e, nullptr, 10) : (1ull << 27);
}

int ensure_weight_stream(tt_graph *g, hipStream_t s, uint32_t bin) {
    std::lock_guard<std::mutex> lock(g->init_mu);
    const uint32_t have = g->ws_low.load(std::memory_order_acquire);
    if (have <= bin) return TT_OK;
    const uint64_t m = g->m;
    int rc;
    if (!g->ws_src) {
        uint32_t *ws[5] = {};
        for (int i = 0; i < (g->hmx ? 5 : 4); i++)
            if ((rc = dev_alloc(g, (void **)&ws[i], (m + 1) * 4))) {
                for (auto &x : ws) dev_free(g, x, 0);
                return rc;
            }
        if ((rc = dev_alloc(g, (void **)&g->ws_base, WBINS * 8))) {
            for (auto &x : ws) dev_free(g, x, 0);
            return rc;
        }
        HIP_TRY(hipMemcpyAsync(g->ws_base, g->wbase.data(), WBINS * 8, hipMemcpyHostToDevice, s));
        g->ws_hmx = ws[4];
        g->ws_col = ws[1];
        g->ws_wgt = ws[2];
        g->ws_pos = ws[3];
        g->ws_src = ws[0];
    }
    // extend down while the placed prefix is under twice the requested one
    const auto prefix = [&](uint32_t b) { return g->wbase[b] + g->whist[b]; };
    const uint64_t want = std::min<uint64_t>(m, std::max<uint64_t>(WS_GROW * prefix(bin), m / WS_MIN_FRAC));
    uint32_t lo = bin;
    while (lo > 0 && prefix(lo) < want) lo--;
    if (m <= ws_all_at_once()) lo = 0;
    Scratch S;
    S.stream = s;
    unsigned long long *bincur = nullptr;
    if ((rc = S.get((void **)&bincur, WBINS * 8))) return rc;
    HIP_TRY(hipMemsetAsync(bincur, 0, WBINS * 8, s));
    if (m && m <= ws_all_at_once()) {
        const uint64_t per = 256ull * PLACE_ITEMS;
        k_place_entries<<<(unsigned)((m + per - 1) / per), 256, 0, s>>>(g->osrc, g->col, g->wgt, m, lo, have, g->ws_base,
                                                                        bincur, g->hmx, g->ws_src, g->ws_col,
                                                                        g->ws_wgt, g->ws_pos, g->ws_hmx);
    } else if (m) {
        const uint64_t per = 256ull * PLACE_ROWS;
        k_place_row_runs<<<(unsigned)(((uint64_t)g->n + per - 1) / per), 256, 0, s>>>(
            g->rstart, g->rlen, g->maxw, g->n, g->wcol, g->wwgt, g->wpos, lo, have, g->ws_base, bincur, g->hmx,
            g->ws_src, g->ws_col, g->ws_wgt, g->ws_pos, g->ws_hmx);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s)); // complete before other streams may see it
    g->ws_low.store(lo, std::memory_order_release);
    return TT_OK;
}

// The transpose of the oriented CSR (built once, on the first subset query).
int ensure_in_csr(tt_graph *g, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g->init_mu);
    if (g->irstart) return TT_OK;
    const uint64_t nn = (uint64_t)g->n + 1, m = g->m;
    int rc;
    Scratch S;
    S.stream = s;
    uint32_t *indeg = nullptr, *cursor = nullptr;
    uint64_t *irstart = nullptr;
    uint32_t *itail = nullptr;
    if ((rc = S.get((void **)&indeg, nn * 4)) || (rc = S.get((void **)&cursor, nn * 4)) ||
        (rc = dev_alloc(g, (void **)&irstart, (nn + 1) * 8)) || (rc = dev_alloc(g, (void **)&itail, (m + 1) * 4))) {
        dev_free(g, irstart, 0);
        dev_free(g, itail, 0);
        return rc;
    }
    HIP_TRY(hipMemsetAsync(indeg, 0, nn * 4, s));
    HIP_TRY(hipMemsetAsync(cursor, 0, nn * 4, s));
    if (m) k_indeg<<<grid_for(m), 256, 0, s>>>(g->col, m, indeg);
    if ((rc = exclusive_scan_u32_to_u64(indeg, irstart, nn, s, nullptr))) return rc;
    if (m) k_in_scatter<<<grid_for(m), 256, 0, s>>>(g->col, g->osrc, m, irstart, cursor, itail);
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    g->irstart = irstart;
    g->itail = itail;
    return TT_OK;
}

static int load_common(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                       void *stream, bool host, tt_graph **out) {
    if (!out) return fail(TT_E_ARG, "out is NULL");
    *out = nullptr;
    if (m && (!src || !dst || !w)) return fail(TT_E_ARG, "src, dst or w is NULL");
    if (n > 0xFFFFFFFEu) return fail(TT_E_TOO_LARGE, "n must be <= 2^32 - 2");
    if (m > 0xFFFFFFFEull) return fail(TT_E_TOO_LARGE, "m must be <= 2^32 - 2");
    tt_graph *g = new (std::nothrow) tt_graph();
    if (!g) return fail(TT_E_NOMEM, "host allocation failed");
    g->n = n;
    g->m = m;
    (void)hipGetDevice(&g->device);
    if (stream) g->stream = (hipStream_t)stream;
    else {
        hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { delete g; return fail(TT_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e)); }
        g->owns_stream = true;
    }
    g->q.stream = g->stream;
    int rc = TT_OK;
    const uint32_t *ds = src, *dd = dst, *dw = w;
    uint32_t *copy = nullptr;
    if (host && m) {
        rc = dev_alloc(nullptr, (void **)&copy, 3 * m * 4);
        if (!rc) {
            hipError_t e = hipMemcpyAsync(copy, src, m * 4, hipMemcpyHostToDevice, g->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(copy + m, dst, m * 4, hipMemcpyHostToDevice, g->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(copy + 2 * m, w, m * 4, hipMemcpyHostToDevice, g->stream);
            if (e != hipSuccess) rc = fail(TT_E_DEVICE, std::string("host-to-device copy: ") + hipGetErrorString(e));
            ds = copy; dd = copy + m; dw = copy + 2 * m;
        }
    }
    if (!rc) rc = build_csr(g, ds, dd, dw);
    if (copy) { (void)hipStreamSynchronize(g->stream); dev_free(nullptr, copy, 3 * m * 4); }
    if (rc) { graph_free(g); return rc; }
    *out = g;
    set_error("");
    return TT_OK;
}

extern "C" int graph_load(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                          tt_graph **out) {
    return load_common(n, m, src, dst, w, nullptr, true, out);
}

extern "C" int graph_load_device(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                                 void *stream, tt_graph **out) {
    return load_common(n, m, src, dst, w, stream, false, out);
}

extern "C" uint32_t graph_num_vertices(const tt_graph *g) { return g ? g->n : 0; }
extern "C" uint64_t graph_num_edges(const tt_graph *g) { return g ? g->m : 0; }
extern "C" uint64_t graph_device_bytes(const tt_graph *g) { return g ? g->bytes : 0; }

void ctx_release(QueryCtx *q) {
    void *ptrs[] = {q->buf0,    q->buf1,    q->cand,    q->ccnt,    q->spart,    q->dcount, q->dout,
                    q->vflag,   q->vflag2,  q->sub_src, q->sub_col, q->sub_wgt,  q->sub_pos, q->sub_vlist,
                    q->sp_c,    q->sp_w,    q->sp_start, q->sp_cnt,
                    q->heavy,   q->nheavy,  q->hpiece};
    for (void *p : ptrs) dev_free(nullptr, p, 0);
    q->buf0 = q->buf1 = nullptr;
    q->cand = nullptr;
    q->ccnt = nullptr;
    q->heavy = nullptr;
    q->nheavy = nullptr;
    q->hpiece = nullptr;
    q->spart = nullptr;
    q->dcount = nullptr;
    q->dout = nullptr;
    q->vflag = q->vflag2 = nullptr;
    q->sub_src = q->sub_col = q->sub_wgt = q->sub_pos = q->sub_vlist = nullptr;
    q->sp_c = q->sp_w = q->sp_start = q->sp_cnt = nullptr;
    q->sub_active = false;
    q->buf_cap = q->cand_cap = q->dout_cap = 0;
    if (q->hcount) (void)hipHostFree(q->hcount);
    q->hcount = nullptr;
    if (q->hout) (void)hipHostFree(q->hout);
    q->hout = nullptr;
    for (auto &e : q->ev)
        if (e) { (void)hipEventDestroy(e); e = nullptr; }
    for (auto &e : q->band_ev)
        if (e) (void)hipEventDestroy(e);
    q->band_ev.clear();
}

extern "C" void graph_free(tt_graph *g) {
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    release(g);
    if (g->owns_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}
