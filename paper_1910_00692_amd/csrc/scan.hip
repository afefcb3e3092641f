// scan.hip — device prefix sums (reduce, scan block sums, rescan), used for CSR row offsets
// and for the cumulative edge weights of weighted edge sampling (Alg. 3).
#include "common.h"
#include "scan.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Block-wide exclusive scan of one value per thread (LDS Hillis-Steele; T may be u128).
template <typename T> __device__ T block_excl_scan(T x, T *sh, T *total) {
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int o = 1; o < SCAN_THREADS; o <<= 1) {
        T y = t >= o ? sh[t - o] : T(0);
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    T incl = sh[t];
    *total = sh[SCAN_THREADS - 1];
    __syncthreads();
    return incl - x;
}

template <typename T, typename F> __global__ __launch_bounds__(SCAN_THREADS) void k_reduce(uint64_t n, F f, T *bsum) {
    __shared__ T sh[SCAN_THREADS];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    T acc = 0;
    for (int it = 0; it < SCAN_ITEMS; it++) {
        uint64_t i = base + (uint64_t)it * SCAN_THREADS + threadIdx.x;
        if (i < n) acc += f(i);
    }
    T tot;
    block_excl_scan<T>(acc, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of nb block sums in one block (chunks of SCAN_THREADS with a carry).
template <typename T> __global__ __launch_bounds__(SCAN_THREADS) void k_scan_sums(T *bsum, uint64_t nb) {
    __shared__ T sh[SCAN_THREADS];
    T carry = 0;
    for (uint64_t c = 0; c < nb; c += SCAN_THREADS) {
        uint64_t i = c + threadIdx.x;
        T x = i < nb ? bsum[i] : T(0);
        T tot;
        T ex = block_excl_scan<T>(x, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

template <typename T, typename F>
__global__ __launch_bounds__(SCAN_THREADS) void k_rescan(uint64_t n, F f, const T *bsum, T *out, int inclusive) {
    __shared__ T sh[SCAN_THREADS];
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T acc = 0;
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; it++) {
        uint64_t i = base + it;
        v[it] = i < n ? f(i) : T(0);
        acc += v[it];
    }
    T tot;
    T run = block_excl_scan<T>(acc, sh, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int it = 0; it < SCAN_ITEMS; it++) {
        uint64_t i = base + it;
        if (i < n) {
            if (inclusive) { run += v[it]; out[i] = run; }
            else { out[i] = run; run += v[it]; }
        }
    }
}

struct LoadU32 {
    const uint32_t *p;
    __device__ uint64_t operator()(uint64_t i) const { return p[i]; }
};

template <typename T, typename F> int scan_impl(uint64_t n, F f, T *out, int inclusive, hipStream_t s, tt_graph *g) {
    if (n == 0) return TT_OK;
    const uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    T *bsum = nullptr;
    int rc = dev_alloc(g, (void **)&bsum, nb * sizeof(T));
    if (rc) return rc;
    k_reduce<T, F><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(n, f, bsum);
    k_scan_sums<T><<<1, SCAN_THREADS, 0, s>>>(bsum, nb);
    k_rescan<T, F><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(n, f, bsum, out, inclusive);
    hipError_t e = hipGetLastError();
    (void)hipStreamSynchronize(s);
    dev_free(g, bsum, nb * sizeof(T));
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

int exclusive_scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, hipStream_t s, tt_graph *g) {
    return scan_impl<uint64_t>(n, LoadU32{in}, out, 0, s, g);
}

int inclusive_weight_prefix(tt_graph *g, double q, void *out) {
    if (q == 1.0) return scan_impl<uint64_t>(g->m, PowU64{g->in_w}, (uint64_t *)out, 1, g->stream, g);
    if (q == 2.0 || q == 3.0) return scan_impl<u128>(g->m, PowU128{g->in_w, (int)q}, (u128 *)out, 1, g->stream, g);
    return scan_impl<double>(g->m, PowF64{g->in_w, q}, (double *)out, 1, g->stream, g);
}
