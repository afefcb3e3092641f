// graph.hip — graph_load: validation and the degree-oriented CSR, built on the device.
//
// The brute-force enumerator of Sec. 3 (NodeIterator++) visits each triangle once from its
// vertex of highest degree; the equivalent edge view used here orients every edge from the
// endpoint that is lower in (degree, ID) order to the higher one, so that each triangle
// {a < b < c} (in that order) is found exactly once, at entry a->b, as c in out(a) ∩ out(b).
// Out-degrees are then at most sqrt(2m), which bounds the cost of every intersection.
#include <cstring>
#include <cstdio>
#include <chrono>

#include "common.h"

// ----------------------------------------------------------------------------- errors
static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}
extern "C" const char *tt_last_error(void) { return g_last_error.c_str(); }

int dev_alloc(tt_graph *g, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(TT_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " + hipGetErrorString(e));
    }
    if (g) g->bytes += bytes;
    return TT_OK;
}
void dev_free(tt_graph *g, void *p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    if (g) g->bytes -= (bytes == 0 ? 16 : bytes);
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
    // OR-reduce the wave, one atomic per wave
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

// Rows of at most 64 entries: one wave per row, each lane's rank found by counting.
// Longer rows are queued for k_sort_big_rows.
__global__ __launch_bounds__(256) void k_sort_small_rows(const uint64_t *rowp, uint32_t n, uint32_t *col, uint32_t *wgt,
                                                         uint32_t *eid, uint32_t *big, uint32_t *nbig) {
    const uint64_t row = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const uint64_t b = rowp[row];
    const uint32_t len = (uint32_t)(rowp[row + 1] - b);
    if (len <= 1) return;
    if (len > 64) {
        if (lane == 0) big[atomicAdd(nbig, 1u)] = (uint32_t)row;
        return;
    }
    uint32_t c = 0xFFFFFFFFu, w = 0, e = 0;
    if (lane < (int)len) { c = col[b + lane]; w = wgt[b + lane]; e = eid[b + lane]; }
    uint32_t rank = 0;
    for (uint32_t j = 0; j < len; j++) {
        uint32_t cj = __shfl(c, (int)j, 64);
        rank += (cj < c) || (cj == c && (int)j < lane);
    }
    if (lane < (int)len) { col[b + rank] = c; wgt[b + rank] = w; eid[b + rank] = e; }
}

constexpr int BIG_TILE = 2048;

// One block per long row: bitonic sort of 2048-entry tiles in LDS, then stable merges by
// rank (each element finds its place in the sibling run by binary search).
__global__ __launch_bounds__(256) void k_sort_big_rows(const uint64_t *rowp, const uint32_t *big, uint32_t nbig,
                                                       uint32_t *col, uint32_t *wgt, uint32_t *eid, uint32_t *tcol,
                                                       uint32_t *twgt, uint32_t *teid) {
    __shared__ uint32_t sc[BIG_TILE], sw[BIG_TILE], se[BIG_TILE];
    for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
        const uint32_t row = big[bi];
        const uint64_t b = rowp[row];
        const uint32_t len = (uint32_t)(rowp[row + 1] - b);
        for (uint32_t t0 = 0; t0 < len; t0 += BIG_TILE) {
            const uint32_t tl = min((uint32_t)BIG_TILE, len - t0);
            uint32_t P = 1;
            while (P < tl) P <<= 1;
            for (uint32_t t = threadIdx.x; t < P; t += blockDim.x) {
                if (t < tl) { sc[t] = col[b + t0 + t]; sw[t] = wgt[b + t0 + t]; se[t] = eid[b + t0 + t]; }
                else { sc[t] = 0xFFFFFFFFu; sw[t] = 0; se[t] = 0; }
            }
            __syncthreads();
            for (uint32_t size = 2; size <= P; size <<= 1) {
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                        uint32_t i = 2 * t - (t & (stride - 1)), j = i + stride;
                        bool asc = (i & size) == 0;
                        if ((sc[i] > sc[j]) == asc) {
                            uint32_t x = sc[i]; sc[i] = sc[j]; sc[j] = x;
                            x = sw[i]; sw[i] = sw[j]; sw[j] = x;
                            x = se[i]; se[i] = se[j]; se[j] = x;
                        }
                    }
                    __syncthreads();
                }
            }
            for (uint32_t t = threadIdx.x; t < tl; t += blockDim.x) {
                col[b + t0 + t] = sc[t]; wgt[b + t0 + t] = sw[t]; eid[b + t0 + t] = se[t];
            }
            __syncthreads();
        }
        // merge rounds
        uint32_t *ic = col + b, *iw = wgt + b, *ie = eid + b, *oc = tcol + b, *ow = twgt + b, *oe = teid + b;
        bool in_tmp = false;
        for (uint32_t R = BIG_TILE; R < len; R <<= 1) {
            for (uint32_t x = threadIdx.x; x < len; x += blockDim.x) {
                const uint32_t r = x / R, i = x - r * R, base = (r & ~1u) * R;
                const uint32_t key = ic[x];
                uint32_t lo, hi;
                if ((r & 1u) == 0) { lo = (r + 1) * R; hi = min((r + 2) * R, len); if (lo > len) lo = len; }
                else { lo = (r - 1) * R; hi = r * R; }
                const uint32_t o0 = lo;
                const bool left = (r & 1u) == 0;
                while (lo < hi) { // lower_bound (left run) / upper_bound (right run)
                    uint32_t mid = (lo + hi) >> 1;
                    bool go = left ? (ic[mid] < key) : (ic[mid] <= key);
                    if (go) lo = mid + 1; else hi = mid;
                }
                const uint32_t pos = base + i + (lo - o0);
                oc[pos] = key; ow[pos] = iw[x]; oe[pos] = ie[x];
            }
            __syncthreads();
            uint32_t *t;
            t = ic; ic = oc; oc = t;
            t = iw; iw = ow; ow = t;
            t = ie; ie = oe; oe = t;
            in_tmp = !in_tmp;
        }
        if (in_tmp) {
            for (uint32_t x = threadIdx.x; x < len; x += blockDim.x) { col[b + x] = ic[x]; wgt[b + x] = iw[x]; eid[b + x] = ie[x]; }
        }
        __syncthreads();
    }
}

// One wave per row: tail IDs, input-edge positions, row maximum, duplicate check.
__global__ __launch_bounds__(256) void k_row_post(const uint64_t *rowp, uint32_t n, const uint32_t *col,
                                                  const uint32_t *wgt, const uint32_t *eid, uint32_t *osrc,
                                                  uint32_t *opos, uint32_t *maxw, uint32_t *flags, uint32_t *gmax) {
    const uint64_t row = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    const uint64_t b = rowp[row], e = rowp[row + 1];
    uint32_t mx = 0;
    bool dup = false;
    for (uint64_t t = b + lane; t < e; t += 64) {
        uint32_t c = col[t];
        osrc[t] = (uint32_t)row;
        opos[eid[t]] = (uint32_t)t;
        mx = max(mx, wgt[t]);
        if (t > b && col[t - 1] == c) dup = true;
    }
    mx = wave_max(mx);
    uint64_t anydup = __ballot(dup);
    if (lane == 0) {
        maxw[row] = mx;
        if (mx) atomicMax(&gmax[0], mx);
        if (e > b) atomicMax(&gmax[1], (uint32_t)(e - b));
        if (anydup) atomicOr(flags, F_DUP);
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

void release(tt_graph *g) {
    if (!g) return;
    void *ptrs[] = {g->rowp, g->col, g->wgt, g->osrc, g->eid, g->opos, g->maxw, g->deg, g->buf0, g->buf1, g->dcount,
                    g->dout, g->emark, g->vflag, g->vflag2, g->prefix};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (g->hcount) (void)hipHostFree(g->hcount);
    for (auto &e : g->ev)
        if (e) (void)hipEventDestroy(e);
}

} // namespace

// ----------------------------------------------------------------------------- build
static int build_csr(tt_graph *g, const uint32_t *src, const uint32_t *dst, const uint32_t *w) {
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    hipStream_t s = g->stream;
    int rc;
    uint32_t *flags = nullptr, *outdeg = nullptr, *cursor = nullptr, *big = nullptr, *gmax = nullptr;
    if ((rc = dev_alloc(nullptr, (void **)&flags, 4 * sizeof(uint32_t)))) return rc;
    HIP_TRY(hipMemsetAsync(flags, 0, 4 * sizeof(uint32_t), s));
    if (m) k_validate<<<grid_for(m), 256, 0, s>>>(src, dst, w, m, n, flags);
    uint32_t hf[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hf[0] & F_RANGE) { dev_free(nullptr, flags, 16); return fail(TT_E_VERTEX_RANGE, "an edge endpoint is >= n"); }
    if (hf[0] & F_LOOP) { dev_free(nullptr, flags, 16); return fail(TT_E_SELF_LOOP, "the graph has a self-loop"); }
    if (hf[0] & F_ZERO) { dev_free(nullptr, flags, 16); return fail(TT_E_ZERO_WEIGHT, "an edge weight is 0"); }

    const uint64_t nn = (uint64_t)n + 1;
    if ((rc = dev_alloc(g, (void **)&g->deg, nn * 4)) || (rc = dev_alloc(g, (void **)&g->rowp, (nn + 1) * 8)) ||
        (rc = dev_alloc(g, (void **)&g->maxw, nn * 4)) || (rc = dev_alloc(g, (void **)&g->col, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->wgt, (m + 1) * 4)) || (rc = dev_alloc(g, (void **)&g->osrc, (m + 1) * 4)) ||
        (rc = dev_alloc(g, (void **)&g->eid, (m + 1) * 4)) || (rc = dev_alloc(g, (void **)&g->opos, (m + 1) * 4)) ||
        (rc = dev_alloc(nullptr, (void **)&outdeg, nn * 4)) || (rc = dev_alloc(nullptr, (void **)&cursor, nn * 4)) ||
        (rc = dev_alloc(nullptr, (void **)&big, nn * 4)) || (rc = dev_alloc(nullptr, (void **)&gmax, 16))) {
        dev_free(nullptr, flags, 16); dev_free(nullptr, outdeg, 0); dev_free(nullptr, cursor, 0);
        dev_free(nullptr, big, 0); dev_free(nullptr, gmax, 0);
        return rc;
    }
    HIP_TRY(hipMemsetAsync(g->deg, 0, nn * 4, s));
    HIP_TRY(hipMemsetAsync(outdeg, 0, nn * 4, s));
    HIP_TRY(hipMemsetAsync(cursor, 0, nn * 4, s));
    HIP_TRY(hipMemsetAsync(gmax, 0, 16, s));
    if (m) {
        k_degree<<<grid_for(m), 256, 0, s>>>(src, dst, m, g->deg);
        k_outdeg<<<grid_for(m), 256, 0, s>>>(src, dst, m, g->deg, outdeg);
    }
    rc = exclusive_scan_u32_to_u64(outdeg, g->rowp, nn, s, nullptr); // rowp[n] = m
    if (rc) return rc;
    if (m) k_scatter<<<grid_for(m), 256, 0, s>>>(src, dst, w, m, g->deg, g->rowp, cursor, g->col, g->wgt, g->eid);
    HIP_TRY(hipMemsetAsync(flags + 1, 0, 4, s));
    if (n) k_sort_small_rows<<<(unsigned)(((uint64_t)n + 3) / 4), 256, 0, s>>>(g->rowp, n, g->col, g->wgt, g->eid, big,
                                                                              flags + 1);
    HIP_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint32_t nbig = hf[1];
    if (nbig) {
        uint32_t *t3 = nullptr;
        if ((rc = dev_alloc(nullptr, (void **)&t3, (m + 1) * 12))) return rc;
        unsigned grid = nbig < 4096u ? nbig : 4096u;
        k_sort_big_rows<<<grid, 256, 0, s>>>(g->rowp, big, nbig, g->col, g->wgt, g->eid, t3, t3 + (m + 1),
                                             t3 + 2 * (m + 1));
        HIP_TRY(hipStreamSynchronize(s));
        dev_free(nullptr, t3, (m + 1) * 12);
    }
    if (n) k_row_post<<<(unsigned)(((uint64_t)n + 3) / 4), 256, 0, s>>>(g->rowp, n, g->col, g->wgt, g->eid, g->osrc,
                                                                       g->opos, g->maxw, flags, gmax);
    unsigned long long *hist = nullptr;
    if ((rc = dev_alloc(nullptr, (void **)&hist, WBINS * 8))) return rc;
    HIP_TRY(hipMemsetAsync(hist, 0, WBINS * 8, s));
    if (m) k_weight_hist<<<grid_for(m), 256, 0, s>>>(g->wgt, m, hist);
    g->whist.assign(WBINS, 0);
    uint32_t hm[4];
    HIP_TRY(hipMemcpyAsync(g->whist.data(), hist, WBINS * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hm, gmax, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    g->wmax = hm[0];
    g->max_outdeg = hm[1];
    dev_free(nullptr, hist, WBINS * 8);
    dev_free(nullptr, flags, 16); dev_free(nullptr, outdeg, nn * 4); dev_free(nullptr, cursor, nn * 4);
    dev_free(nullptr, big, nn * 4); dev_free(nullptr, gmax, 16);
    if (hf[0] & F_DUP) return fail(TT_E_DUP_EDGE, "the same unordered vertex pair appears twice");
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
