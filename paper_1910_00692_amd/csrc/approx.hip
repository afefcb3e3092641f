// approx.hip — the paper's approximate methods beside the exact path: the static heavy-light
// algorithm (Alg. 1, Sec. 3).
//
// Alg. 1 keeps the edges heavier than a threshold tau and enumerates the triangles of the
// subgraph they induce: a triangle is found only if all three of its edges are heavy, so the
// answer is the exact top-k of G[H] and an approximation of the top-k of G.  Here G[H] is
// compacted from the resident oriented CSR on the device and answered by the exact path.
#include <cstring>

#include "common.h"

namespace {

// Entries of weight > tau appended to (s, d, w): one ballot and one global atomic per wave.
__global__ __launch_bounds__(256) void k_compact_heavy(const uint32_t *osrc, const uint32_t *col, const uint32_t *wgt,
                                                       uint64_t m, uint32_t tau, uint32_t *s, uint32_t *d, uint32_t *w,
                                                       unsigned long long *count, uint64_t cap) {
    const int lane = threadIdx.x & 63;
    for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~63ull; base < m;
         base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = base + lane;
        const bool keep = e < m && wgt[e] > tau;
        const uint64_t bal = __ballot(keep);
        if (!bal) continue;
        unsigned long long b0 = 0;
        if (lane == 0) b0 = atomicAdd(count, (unsigned long long)__popcll(bal));
        b0 = __shfl(b0, 0, 64);
        const uint64_t slot = b0 + __popcll(bal & ((1ull << lane) - 1ull));
        if (keep && slot < cap) {
            s[slot] = osrc[e];
            d[slot] = col[e];
            w[slot] = wgt[e];
        }
    }
}

} // namespace

extern "C" int shl_topk_triangles(tt_graph *g, uint32_t k, double p, uint32_t tau, tt_triangle *out, uint32_t *n_out,
                                  uint64_t *heavy_edges) {
    if (n_out) *n_out = 0;
    if (heavy_edges) *heavy_edges = 0;
    if (!g || !n_out) return fail(TT_E_ARG, "graph or n_out is NULL");
    if (p != p) return fail(TT_E_ARG, "p is NaN");
    if (k && !out) return fail(TT_E_ARG, "out is NULL");
    if (g->m == 0) { set_error(""); return TT_OK; }
    hipStream_t s = nullptr;
    uint64_t cap = 0;
    {
        // entries in weight bins that can hold a weight > tau bound the heavy count
        const uint32_t b = tau == 0xFFFFFFFFu ? (uint32_t)WBINS : weight_bin(tau + 1);
        for (uint32_t x = b; x < (uint32_t)WBINS; x++) cap += g->whist[x];
    }
    std::lock_guard<std::mutex> lock(g->mu);
    (void)hipSetDevice(g->device);
    s = g->stream;
    uint32_t *buf = nullptr;
    unsigned long long *cnt = nullptr;
    int rc;
    if ((rc = dev_alloc(nullptr, (void **)&buf, (3 * cap + 1) * 4)) ||
        (rc = dev_alloc(nullptr, (void **)&cnt, 256))) {
        dev_free(nullptr, buf, 0);
        return rc;
    }
    struct Free {
        uint32_t *b; unsigned long long *c; hipStream_t s;
        ~Free() { (void)hipStreamSynchronize(s); dev_free(nullptr, b, 0); dev_free(nullptr, c, 0); }
    } guard{buf, cnt, s};
    uint32_t *hs = buf, *hd = buf + cap, *hw = buf + 2 * cap;
    HIP_TRY(hipMemsetAsync(cnt, 0, 8, s));
    const uint64_t blocks = std::min<uint64_t>((g->m + 255) / 256, (uint64_t)num_cus() * 16);
    k_compact_heavy<<<(unsigned)blocks, 256, 0, s>>>(g->osrc, g->col, g->wgt, g->m, tau, hs, hd, hw, cnt, cap);
    HIP_TRY(hipGetLastError());
    unsigned long long mh = 0;
    HIP_TRY(hipMemcpyAsync(&mh, cnt, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (mh > cap) return fail(TT_E_DEVICE, "internal: more heavy entries than the weight histogram allows");
    if (heavy_edges) *heavy_edges = mh;
    if (k == 0 || mh < 3) { set_error(""); return TT_OK; }
    tt_graph *h = nullptr;
    if ((rc = graph_load_device(g->n, mh, hs, hd, hw, s, &h))) return rc;
    rc = topk_triangles(h, k, p, out, n_out);
    graph_free(h);
    if (!rc) set_error("");
    return rc;
}
