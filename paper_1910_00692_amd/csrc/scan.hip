// scan.hip — device prefix sums (reduce, scan block sums, rescan), used for CSR row offsets
// and for the cumulative edge weights of weighted edge sampling (Alg. 3).
#include "common.h"
#include "scan.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// __shfl_up of a 4-, 8- or 16-byte value, one 32-bit word at a time.
template <typename T> __device__ __forceinline__ T shfl_up_words(T x, int o) {
    constexpr int W = sizeof(T) / 4;
    union U {
        T v;
        uint32_t w[W];
    } a, b;
    a.v = x;
#pragma unroll
    for (int i = 0; i < W; i++) b.w[i] = __shfl_up(a.w[i], o, 64);
    return b.v;
}

// Block-wide exclusive scan of one value per thread: a shuffle scan in each wave, then the
// four wave totals through LDS.  *total = the sum over the block.
template <typename T> __device__ T block_excl_scan(T x, T *wtot, T *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = shfl_up_words(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SCAN_THREADS / 64; i++) {
        if (i < w) off += wtot[i];
        tot += wtot[i];
    }
    *total = tot;
    __syncthreads(); // wtot may be reused at once
    return off + incl - x;
}

template <typename T, typename F> __global__ __launch_bounds__(SCAN_THREADS) void k_reduce(uint64_t n, F f, T *bsum) {
    __shared__ T wtot[SCAN_THREADS / 64];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    T acc = 0;
    for (int it = 0; it < SCAN_ITEMS; it++) {
        uint64_t i = base + (uint64_t)it * SCAN_THREADS + threadIdx.x;
        if (i < n) acc += f(i);
    }
    T tot;
    block_excl_scan<T>(acc, wtot, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of nb block sums in one block (chunks of SCAN_THREADS with a carry).
template <typename T> __global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(T *bsum, uint64_t nb) {
    __shared__ T wtot[SCAN_THREADS / 64];
    T carry = 0;
    for (uint64_t c = 0; c < nb; c += SCAN_THREADS) {
        uint64_t i = c + threadIdx.x;
        T x = i < nb ? bsum[i] : T(0);
        T tot;
        T ex = block_excl_scan<T>(x, wtot, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

// The tile passes through LDS so that global loads and stores are coalesced while each thread
// scans SCAN_ITEMS consecutive elements (one pad slot per 8 keeps the strided LDS reads apart).
__device__ __forceinline__ uint32_t scan_pad(uint32_t j) { return j + (j >> 3); }

template <typename T, typename F>
__global__ __launch_bounds__(SCAN_THREADS) void k_rescan(uint64_t n, F f, const T *bsum, T *out, int inclusive) {
    __shared__ T tile[SCAN_TILE + SCAN_TILE / 8];
    __shared__ T wtot[SCAN_THREADS / 64];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; it++) {
        const uint32_t j = (uint32_t)it * SCAN_THREADS + threadIdx.x;
        tile[scan_pad(j)] = base + j < n ? f(base + j) : T(0);
    }
    __syncthreads();
    T v[SCAN_ITEMS];
    T acc = 0;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; it++) {
        v[it] = tile[scan_pad(threadIdx.x * SCAN_ITEMS + it)];
        acc += v[it];
    }
    T tot;
    T run = block_excl_scan<T>(acc, wtot, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; it++) {
        T r;
        if (inclusive) { run += v[it]; r = run; }
        else { r = run; run += v[it]; }
        tile[scan_pad(threadIdx.x * SCAN_ITEMS + it)] = r; // this thread's own slots
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; it++) {
        const uint32_t j = (uint32_t)it * SCAN_THREADS + threadIdx.x;
        if (base + j < n) out[base + j] = tile[scan_pad(j)];
    }
}

struct LoadU32 {
    const uint32_t *p;
    __device__ uint64_t operator()(uint64_t i) const { return p[i]; }
};
struct LoadF64 {
    const double *p;
    __device__ double operator()(uint64_t i) const { return p[i]; }
};

// With tmp (>= scan_tmp_bytes(n) bytes, caller-owned) the scan is only enqueued; without it the
// block sums are allocated here and the stream is synchronised before they are freed.
template <typename T, typename F>
int scan_impl(uint64_t n, F f, T *out, int inclusive, hipStream_t s, tt_graph *g, void *tmp) {
    if (n == 0) return TT_OK;
    const uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    T *bsum = (T *)tmp;
    if (!bsum) {
        int rc = dev_alloc(g, (void **)&bsum, nb * sizeof(T));
        if (rc) return rc;
    }
    k_reduce<T, F><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(n, f, bsum);
    k_scan_sums<T><<<1, SCAN_THREADS, 0, s>>>(bsum, nb);
    k_rescan<T, F><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(n, f, bsum, out, inclusive);
    hipError_t e = hipGetLastError();
    if (!tmp) {
        (void)hipStreamSynchronize(s);
        dev_free(g, bsum, nb * sizeof(T));
    }
    if (e != hipSuccess) return fail(TT_E_DEVICE, std::string("scan launch: ") + hipGetErrorString(e));
    return TT_OK;
}

// w^q of input edge e (q = 1, 2, 3 exact)
struct PowU128 {
    const uint32_t *w_in;
    int q;
    __device__ u128 operator()(uint64_t e) const {
        u128 w = w_in[e], t = w;
        if (q >= 2) t *= w;
        if (q >= 3) t *= w;
        return t;
    }
};
struct PowU64 {
    const uint32_t *w_in;
    __device__ uint64_t operator()(uint64_t e) const { return w_in[e]; }
};
struct PowF64 {
    const uint32_t *w_in;
    double q;
    __device__ double operator()(uint64_t e) const { return pow((double)w_in[e], q); }
};

} // namespace

uint64_t scan_tmp_bytes(uint64_t n) { return ((n + SCAN_TILE - 1) / SCAN_TILE) * 16 + 16; }

int exclusive_scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, hipStream_t s, tt_graph *g, void *tmp) {
    return scan_impl<uint64_t>(n, LoadU32{in}, out, 0, s, g, tmp);
}

int inclusive_weight_prefix(tt_graph *g, double q, void *out, void *tmp) {
    if (q == 1.0) return scan_impl<uint64_t>(g->m, PowU64{g->in_w}, (uint64_t *)out, 1, g->stream, g, tmp);
    if (q == 2.0 || q == 3.0)
        return scan_impl<u128>(g->m, PowU128{g->in_w, (int)q}, (u128 *)out, 1, g->stream, g, tmp);
    return scan_impl<double>(g->m, PowF64{g->in_w, q}, (double *)out, 1, g->stream, g, tmp);
}

int inclusive_scan_f64(const double *in, double *out, uint64_t n, hipStream_t s, void *tmp) {
    return scan_impl<double>(n, LoadF64{in}, out, 1, s, nullptr, tmp);
}
