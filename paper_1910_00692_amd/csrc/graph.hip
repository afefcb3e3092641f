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

// Device memory comes from a process-wide cache of freed blocks (exact rounded sizes), so that
// repeated loads and queries do not pay for hipMalloc/hipFree.  Blocks are only returned to the
// cache after the work that used them has completed on its stream.
namespace {
std::mutex g_pool_mu;
std::multimap<size_t, void *> g_pool;         // free blocks by size
std::unordered_map<void *, size_t> g_live;    // size of every block handed out
size_t g_pool_bytes = 0;
constexpr size_t POOL_CAP = 16ull << 30;

size_t round_size(size_t b) {
    if (b == 0) b = 16;
    if (b <= (1u << 20)) return (b + 255) & ~(size_t)255;
    size_t p2 = 1;
    while (p2 < b) p2 <<= 1;
    const size_t step = p2 >> 4;
    return (b + step - 1) / step * step;
}

void pool_release_all() {
    for (auto &kv : g_pool) (void)hipFree(kv.second);
    g_pool.clear();
    g_pool_bytes = 0;
}
} // namespace

int dev_alloc(tt_graph *g, void **p, size_t bytes) {
    *p = nullptr;
    const size_t sz = round_size(bytes);
    std::lock_guard<std::mutex> lock(g_pool_mu);
    auto it = g_pool.find(sz);
    if (it != g_pool.end()) {
        *p = it->second;
        g_pool.erase(it);
        g_pool_bytes -= sz;
    } else {
        hipError_t e = hipMalloc(p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            pool_release_all();
            e = hipMalloc(p, sz);
        }
        if (e != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return fail(TT_E_NOMEM, "hipMalloc(" + std::to_string(sz) + " bytes) failed: " + hipGetErrorString(e));
        }
    }
    g_live[*p] = sz;
    if (g) g->bytes += sz;
    return TT_OK;
}

// Returns p to the cache; the caller guarantees no queued work still uses it.
void dev_free(tt_graph *g, void *p, size_t) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_pool_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    const size_t sz = it->second;
    g_live.erase(it);
    if (g) g->bytes -= sz;
    if (g_pool_bytes + sz <= POOL_CAP) {
        g_pool.insert({sz, p});
        g_pool_bytes += sz;
    } else {
        (void)hipFree(p);
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

__global__ __launch_bounds__(256) void k_validate(const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                                                  uint64_t m, uint32_t n, uint32_t *flags) {
    uint32_t f = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t a = src[e], b = dst[e];
        if (a >= n || b >= n) f |= F_RANGE;
        else if (a == b) f |= F_LOOP;
        if (w[e] == 0) f |= F_ZERO;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) f |= __shfl_xor(f, o, 64);
    if ((threadIdx.x & 63) == 0 && f) atomicOr(flags, f);
}

__global__ __launch_bounds__(256) void k_degree(const uint32_t *src, const uint32_t *dst, uint64_t m, uint32_t *deg) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        atomicAdd(&deg[src[e]], 1u);
        atomicAdd(&deg[dst[e]], 1u);
    }
}

// tail of the oriented edge: the endpoint lower in (degree, ID) order
__device__ inline void orient(uint32_t a, uint32_t b, const uint32_t *deg, uint32_t &tail, uint32_t &head) {
    uint32_t da = deg[a], db = deg[b];
    bool a_low = da < db || (da == db && a < b);
    tail = a_low ? a : b;
    head = a_low ? b : a;
}

__global__ __launch_bounds__(256) void k_outdeg(const uint32_t *src, const uint32_t *dst, uint64_t m,
                                                const uint32_t *deg, uint32_t *outdeg) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t t, h;
        orient(src[e], dst[e], deg, t, h);
        atomicAdd(&outdeg[t], 1u);
    }
}

__global__ __launch_bounds__(256) void k_scatter(const uint32_t *src, const uint32_t *dst, const uint32_t *w, uint64_t m,
                                                 const uint32_t *deg, const uint64_t *rowp, uint32_t *cursor,
                                                 uint32_t *col, uint32_t *wgt, uint32_t *eid) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t t, h;
        orient(src[e], dst[e], deg, t, h);
        uint64_t pos = rowp[t] + atomicAdd(&cursor[t], 1u);
        col[pos] = h;
        wgt[pos] = w[e];
        eid[pos] = (uint32_t)e;
    }
}

// Segmented sort of every row by key K (ascending), carrying up to two u32 payloads.
// Rows of at most 64 entries: one wave per row, each lane's rank found by counting.
// Longer rows are queued for k_sort_big_rows.
template <typename K>
__global__ __launch_bounds__(256) void k_sort_small_rows(const uint64_t *rstart, const uint32_t *rlen, uint32_t n,
                                                         K *key, uint32_t *p1, uint32_t *p2, uint32_t *big,
                                                         uint32_t *nbig) {
    const uint64_t row = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const uint64_t b = rstart[row];
    const uint32_t len = rlen[row];
    if (len <= 1) return;
    if (len > 64) {
        if (lane == 0) big[atomicAdd(nbig, 1u)] = (uint32_t)row;
        return;
    }
    K c = ~K(0);
    uint32_t x = 0, y = 0;
    if (lane < (int)len) {
        c = key[b + lane];
        x = p1[b + lane];
        if (p2) y = p2[b + lane];
    }
    uint32_t rank = 0;
    for (uint32_t j = 0; j < len; j++) {
        K cj = __shfl(c, (int)j, 64);
        rank += (cj < c) || (cj == c && (int)j < lane);
    }
    if (lane < (int)len) {
        key[b + rank] = c;
        p1[b + rank] = x;
        if (p2) p2[b + rank] = y;
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

// Row maxima and the duplicate check (rows already sorted by head ID).  Grid-stride waves
// keep running maxima in registers and issue one atomic per wave at the end.
__global__ __launch_bounds__(256) void k_row_max(const uint64_t *rstart, const uint32_t *rlen, uint32_t n,
                                                 const uint32_t *col, const uint32_t *wgt, uint32_t *maxw,
                                                 uint32_t *flags, uint32_t *gmax) {
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t gw = 0, gd = 0;
    bool dup = false;
    for (uint64_t row = wave; row < n; row += nwaves) {
        const uint64_t b = rstart[row];
        const uint32_t len = rlen[row];
        uint32_t mx = 0;
        for (uint32_t t = lane; t < len; t += 64) {
            mx = max(mx, wgt[b + t]);
            if (t > 0 && col[b + t - 1] == col[b + t]) dup = true;
        }
        mx = wave_max(mx);
        if (lane == 0) maxw[row] = mx;
        gw = max(gw, mx);
        gd = max(gd, len);
    }
    const uint64_t anydup = __ballot(dup);
    if (lane == 0) {
        if (gw) atomicMax(&gmax[0], gw);
        if (gd) atomicMax(&gmax[1], gd);
        if (anydup) atomicOr(flags, F_DUP);
    }
}

// hb[u] = max(maxw[u], maxw[v] for v in out(u))
__global__ __launch_bounds__(256) void k_row_bound(const uint64_t *rstart, const uint32_t *rlen, uint32_t n,
                                                   const uint32_t *col, const uint32_t *maxw, uint32_t *hb) {
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t row = wave; row < n; row += nwaves) {
        const uint64_t b = rstart[row];
        const uint32_t len = rlen[row];
        uint32_t mx = 0;
        for (uint32_t t = lane; t < len; t += 64) mx = max(mx, maxw[col[b + t]]);
        mx = wave_max(mx);
        if (lane == 0) hb[row] = max(mx, maxw[row]);
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

// Copies every row to its new start; builds the weight-sorted copy's keys.
__global__ __launch_bounds__(256) void k_move_rows(const uint64_t *ostart, const uint64_t *rstart, const uint32_t *rlen,
                                                   uint32_t n, const uint32_t *ocol, const uint32_t *owgt,
                                                   const uint32_t *oeid, uint32_t *col, uint32_t *wgt, uint32_t *eid,
                                                   uint64_t *wkey, uint32_t *wpos) {
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t row = wave; row < n; row += nwaves) {
        const uint64_t a = ostart[row], b = rstart[row];
        const uint32_t len = rlen[row];
        for (uint32_t t = lane; t < len; t += 64) {
            const uint32_t c = ocol[a + t], w = owgt[a + t];
            col[b + t] = c;
            wgt[b + t] = w;
            eid[b + t] = oeid[a + t];
            wkey[b + t] = ((uint64_t)(~w) << 32) | c; // ascending key = weight descending, then ID
            wpos[b + t] = (uint32_t)(b + t);
        }
    }
}

__global__ __launch_bounds__(256) void k_split_keys(const uint64_t *wkey, uint64_t m, uint32_t *wcol, uint32_t *wwgt) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = wkey[e];
        wcol[e] = (uint32_t)k;
        wwgt[e] = ~(uint32_t)(k >> 32);
    }
}

// Tails and input-edge positions of the final layout.
__global__ __launch_bounds__(256) void k_row_post(const uint64_t *rstart, const uint32_t *rlen, uint32_t n,
                                                  const uint32_t *eid, uint32_t *osrc, uint32_t *opos) {
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t row = wave; row < n; row += nwaves) {
        const uint64_t b = rstart[row];
        const uint32_t len = rlen[row];
        for (uint32_t t = lane; t < len; t += 64) {
            osrc[b + t] = (uint32_t)row;
            opos[eid[b + t]] = (uint32_t)(b + t);
        }
    }
}

// Entries grouped by descending weight_bin(weight): LDS offsets inside the block, one global
// atomic per (block, non-empty bin) to reserve the block's range inside the bin.
__global__ __launch_bounds__(256) void k_place_entries(const uint32_t *osrc, const uint32_t *col, const uint32_t *wgt,
                                                       uint64_t m, const unsigned long long *binbase,
                                                       unsigned long long *bincur, uint32_t *ws_src, uint32_t *ws_col,
                                                       uint32_t *ws_wgt, uint32_t *ws_pos) {
    __shared__ uint32_t lc[WBINS];
    __shared__ unsigned long long lb[WBINS];
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x) lc[t] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * blockDim.x * PLACE_ITEMS;
    uint32_t off[PLACE_ITEMS];
#pragma unroll
    for (int it = 0; it < PLACE_ITEMS; it++) {
        const uint64_t e = base + (uint64_t)it * blockDim.x + threadIdx.x;
        off[it] = 0;
        if (e < m) off[it] = atomicAdd(&lc[weight_bin(wgt[e])], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x)
        if (lc[t]) lb[t] = binbase[t] + atomicAdd(&bincur[t], (unsigned long long)lc[t]);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PLACE_ITEMS; it++) {
        const uint64_t e = base + (uint64_t)it * blockDim.x + threadIdx.x;
        if (e < m) {
            const uint32_t w = wgt[e];
            const uint64_t d = lb[weight_bin(w)] + off[it];
            ws_src[d] = osrc[e];
            ws_col[d] = col[e];
            ws_wgt[d] = w;
            ws_pos[d] = (uint32_t)e;
        }
    }
}

__global__ __launch_bounds__(256) void k_weight_hist(const uint32_t *wgt, uint64_t m, unsigned long long *hist) {
    __shared__ uint32_t h[WBINS];
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x) h[t] = 0;
    __syncthreads();
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[weight_bin(wgt[e])], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < WBINS; t += blockDim.x)
        if (h[t]) atomicAdd(&hist[t], (unsigned long long)h[t]);
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
    void *ptrs[] = {g->rstart, g->rlen, g->col,    g->wgt,    g->osrc,   g->eid,   g->opos,  g->wcol,
                    g->wwgt,   g->wpos, g->maxw,   g->hb,     g->deg,    g->buf0,  g->buf1,  g->dcount,
                    g->dout,   g->emark, g->vflag, g->vflag2, g->ws_src, g->ws_col, g->ws_wgt, g->ws_pos, g->cand, g->ccnt, g->spart};
    for (void *p : ptrs) dev_free(g, p, 0);
    for (auto &t : g->tables) {
        dev_free(g, t.prefix, 0);
        dev_free(g, t.guide, 0);
    }
    if (g->hcount) (void)hipHostFree(g->hcount);
    for (auto &e : g->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : g->band_ev)
        if (e) (void)hipEventDestroy(e);
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

template <typename K>
int sort_rows(tt_graph *g, Scratch &S, const uint64_t *rstart, const uint32_t *rlen, K *key, uint32_t *p1, uint32_t *p2,
              uint32_t *big, uint32_t *nbig_dev) {
    hipStream_t s = g->stream;
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    HIP_TRY(hipMemsetAsync(nbig_dev, 0, 4, s));
    if (n) k_sort_small_rows<K><<<(unsigned)(((uint64_t)n + 3) / 4), 256, 0, s>>>(rstart, rlen, n, key, p1, p2, big,
                                                                                 nbig_dev);
    uint32_t nbig = 0;
    HIP_TRY(hipMemcpyAsync(&nbig, nbig_dev, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (nbig) {
        K *tk = nullptr;
        uint32_t *t12 = nullptr;
        int rc;
        if ((rc = S.get((void **)&tk, (m + 1) * sizeof(K))) || (rc = S.get((void **)&t12, 2 * (m + 1) * 4))) return rc;
        unsigned grid = nbig < 4096u ? nbig : 4096u;
        k_sort_big_rows<K><<<grid, 256, 0, s>>>(rstart, rlen, big, nbig, key, p1, p2, tk, t12, t12 + (m + 1));
        HIP_TRY(hipStreamSynchronize(s));
        S.drop(tk);
        S.drop(t12);
    }
    HIP_TRY(hipGetLastError());
    return TT_OK;
}

} // namespace

// ----------------------------------------------------------------------------- build
static int build_csr(tt_graph *g, const uint32_t *src, const uint32_t *dst, const uint32_t *w) {
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    hipStream_t s = g->stream;
    int rc;
    Scratch S;
    S.stream = s;
    uint32_t *flags = nullptr, *outdeg = nullptr, *cursor = nullptr, *big = nullptr, *gmax = nullptr;
    if ((rc = S.get((void **)&flags, 16))) return rc;
    HIP_TRY(hipMemsetAsync(flags, 0, 16, s));
    if (m) k_validate<<<grid_for(m), 256, 0, s>>>(src, dst, w, m, n, flags);
    uint32_t hf[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf[0] & F_RANGE) return fail(TT_E_VERTEX_RANGE, "an edge endpoint is >= n");
    if (hf[0] & F_LOOP) return fail(TT_E_SELF_LOOP, "the graph has a self-loop");
    if (hf[0] & F_ZERO) return fail(TT_E_ZERO_WEIGHT, "an edge weight is 0");

    const uint64_t nn = (uint64_t)n + 1;
    uint64_t *rowp0 = nullptr;
    uint32_t *col0 = nullptr, *wgt0 = nullptr, *eid0 = nullptr;
    if ((rc = dev_alloc(g, (void **)&g->deg, nn * 4)) || (rc = dev_alloc(g, (void **)&g->rstart, nn * 8)) ||
        (rc = dev_alloc(g, (void **)&g->rlen, nn * 4)) || (rc = dev_alloc(g, (void **)&g->maxw, nn * 4)) ||
        (rc = dev_alloc(g, (void **)&g->hb, nn * 4)) || (rc = dev_alloc(g, (void **)&g->col, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->wgt, (m + 1) * 4)) || (rc = dev_alloc(g, (void **)&g->osrc, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->eid, (m + 1) * 4)) || (rc = dev_alloc(g, (void **)&g->opos, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->wcol, (m + 1) * 4)) || (rc = dev_alloc(g, (void **)&g->wwgt, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->wpos, (m + 1) * 4)) || (rc = S.get((void **)&outdeg, nn * 4)) ||
        (rc = S.get((void **)&cursor, nn * 4)) || (rc = S.get((void **)&big, nn * 4)) ||
        (rc = S.get((void **)&gmax, 16)) || (rc = S.get((void **)&rowp0, (nn + 1) * 8)) ||
        (rc = S.get((void **)&col0, (m + 1) * 4)) || (rc = S.get((void **)&wgt0, (m + 1) * 4)) ||
        (rc = S.get((void **)&eid0, (m + 1) * 4)))
        return rc;
    HIP_TRY(hipMemsetAsync(g->deg, 0, nn * 4, s));
    HIP_TRY(hipMemsetAsync(outdeg, 0, nn * 4, s));
    HIP_TRY(hipMemsetAsync(cursor, 0, nn * 4, s));
    HIP_TRY(hipMemsetAsync(gmax, 0, 16, s));
    if (m) {
        k_degree<<<grid_for(m), 256, 0, s>>>(src, dst, m, g->deg);
        k_outdeg<<<grid_for(m), 256, 0, s>>>(src, dst, m, g->deg, outdeg);
    }
    // rows in vertex order first: rowp0[n] = m
    if ((rc = exclusive_scan_u32_to_u64(outdeg, rowp0, nn, s, nullptr))) return rc;
    if (m) k_scatter<<<grid_for(m), 256, 0, s>>>(src, dst, w, m, g->deg, rowp0, cursor, col0, wgt0, eid0);
    HIP_TRY(hipMemcpyAsync(g->rlen, outdeg, nn * 4, hipMemcpyDeviceToDevice, s));
    if ((rc = sort_rows<uint32_t>(g, S, rowp0, g->rlen, col0, wgt0, eid0, big, flags + 1))) return rc;
    if (n) {
        k_row_max<<<wave_grid(n), 256, 0, s>>>(rowp0, g->rlen, n, col0, wgt0, g->maxw, flags, gmax);
        k_row_bound<<<wave_grid(n), 256, 0, s>>>(rowp0, g->rlen, n, col0, g->maxw, g->hb);
    }
    // layout by descending weight_bin(hb)
    unsigned long long *ecnt = nullptr, *bincur = nullptr, *binbase = nullptr;
    if ((rc = S.get((void **)&ecnt, WBINS * 8)) || (rc = S.get((void **)&bincur, WBINS * 8)) ||
        (rc = S.get((void **)&binbase, WBINS * 8)))
        return rc;
    HIP_TRY(hipMemsetAsync(ecnt, 0, WBINS * 8, s));
    HIP_TRY(hipMemsetAsync(bincur, 0, WBINS * 8, s));
    if (n) k_bin_entries<<<grid_for(n), 256, 0, s>>>(g->hb, g->rlen, n, ecnt);
    g->ebin.assign(WBINS, 0);
    g->ebase.assign(WBINS, 0);
    HIP_TRY(hipMemcpyAsync(g->ebin.data(), ecnt, WBINS * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf[0] & F_DUP) return fail(TT_E_DUP_EDGE, "the same unordered vertex pair appears twice");
    {
        uint64_t run = 0;
        for (int b = WBINS - 1; b >= 0; b--) { g->ebase[b] = run; run += g->ebin[b]; }
    }
    HIP_TRY(hipMemcpyAsync(binbase, g->ebase.data(), WBINS * 8, hipMemcpyHostToDevice, s));
    if (n) {
        const uint64_t per = 256ull * PLACE_ITEMS;
        k_place_rows<<<(unsigned)(((uint64_t)n + per - 1) / per), 256, 0, s>>>(g->hb, g->rlen, n, binbase, bincur, g->rstart);
    }
    uint64_t *wkey = nullptr;
    if ((rc = S.get((void **)&wkey, (m + 1) * 8))) return rc;
    if (n) k_move_rows<<<wave_grid(n), 256, 0, s>>>(rowp0, g->rstart, g->rlen, n, col0, wgt0, eid0, g->col, g->wgt,
                                                    g->eid, wkey, g->wpos);
    S.drop(col0);
    S.drop(wgt0);
    S.drop(eid0);
    if ((rc = sort_rows<uint64_t>(g, S, g->rstart, g->rlen, wkey, g->wpos, nullptr, big, flags + 1))) return rc;
    if (m) k_split_keys<<<grid_for(m), 256, 0, s>>>(wkey, m, g->wcol, g->wwgt);
    if (n) k_row_post<<<wave_grid(n), 256, 0, s>>>(g->rstart, g->rlen, n, g->eid, g->osrc, g->opos);
    unsigned long long *hist = nullptr;
    if ((rc = S.get((void **)&hist, WBINS * 8))) return rc;
    HIP_TRY(hipMemsetAsync(hist, 0, WBINS * 8, s));
    if (m) k_weight_hist<<<grid_for(m), 256, 0, s>>>(g->wgt, m, hist);
    g->whist.assign(WBINS, 0);
    uint32_t hm[4];
    HIP_TRY(hipMemcpyAsync(g->whist.data(), hist, WBINS * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hm, gmax, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    g->wmax = hm[0];
    g->max_outdeg = hm[1];
    // the weight-ordered stream of entries
    g->wbase.assign(WBINS, 0);
    {
        uint64_t run = 0;
        for (int b = WBINS - 1; b >= 0; b--) { g->wbase[b] = run; run += g->whist[b]; }
    }
    if ((rc = dev_alloc(g, (void **)&g->ws_src, (m + 1) * 4)) || (rc = dev_alloc(g, (void **)&g->ws_col, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->ws_wgt, (m + 1) * 4)) || (rc = dev_alloc(g, (void **)&g->ws_pos, (m + 1) * 4)))
        return rc;
    HIP_TRY(hipMemcpyAsync(binbase, g->wbase.data(), WBINS * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(bincur, 0, WBINS * 8, s));
    if (m) {
        const uint64_t per = 256ull * PLACE_ITEMS;
        k_place_entries<<<(unsigned)((m + per - 1) / per), 256, 0, s>>>(g->osrc, g->col, g->wgt, m, binbase, bincur,
                                                                        g->ws_src, g->ws_col, g->ws_wgt, g->ws_pos);
    }
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
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

extern "C" void graph_free(tt_graph *g) {
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    release(g);
    if (g->owns_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}
