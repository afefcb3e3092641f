/*
 * topktri.h — top-k weighted triangles on AMD MI355X (gfx950).
 *
 * Problem (Kumar, Liu, Charikar, Benson, "Retrieving Top Weighted Triangles in Graphs",
 * WSDM 2020, Sec. 1): G = (V, E, w) is a simple undirected graph with positive edge
 * weights.  The weight of triangle (i, j, l) is the generalized p-mean of its three edge
 * weights (Eq. 1):  m_p = [ (w_ij^p + w_jl^p + w_il^p) / 3 ]^(1/p),  with the limits named
 * right after Eq. 1: p = 0 is the geometric mean, p = +inf the maximum, p = -inf the minimum.
 * A query returns the k heaviest triangles.
 *
 * Conventions shared by every entry point
 *   - Vertex IDs are uint32 in [0, n); n <= 2^32 - 2.  Weights are uint32 >= 1.
 *   - Results are sorted by score descending, then by (i, j, l) ascending, where
 *     i < j < l are the caller's original vertex IDs.  If the graph (or the admitted set)
 *     holds T < k triangles, all T are returned and *n_out = T.
 *   - For p in {-inf, 0, 1, 2, +inf} the order is decided by exact integer arithmetic
 *     (min, product, sum, sum of squares, max); for any other p by the FP64 value of m_p.
 *     The returned score is the FP64 value of m_p.
 *   - Every function returns an int status (TT_OK = 0, negative on error).  No function
 *     aborts, throws or exits.  On error, *n_out (if given) is set to 0 and other outputs
 *     are untouched.  tt_last_error() returns a message for the calling thread.
 *   - Host pointers are copied before the call returns and never retained.
 *   - A graph is immutable after loading.  Queries on one graph from several host threads
 *     are serialised internally.
 */
#ifndef TOPKTRI_H
#define TOPKTRI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque handle; owns all device memory of one loaded graph. */
typedef struct tt_graph tt_graph;

/* One result triangle: original vertex IDs i < j < l and the FP64 p-mean.  24 bytes. */
typedef struct {
    uint32_t i, j, l, _pad;
    double score;
} tt_triangle;

enum {
    TT_OK = 0,
    TT_E_ARG = -1,          /* NULL pointer, NaN p, bad size */
    TT_E_SELF_LOOP = -2,    /* an edge (v, v) */
    TT_E_DUP_EDGE = -3,     /* the same unordered pair twice */
    TT_E_ZERO_WEIGHT = -4,  /* a weight of 0 (weights must be positive, Sec. 1) */
    TT_E_VERTEX_RANGE = -5, /* an endpoint >= n */
    TT_E_NOMEM = -6,        /* device or host allocation failed */
    TT_E_DEVICE = -7,       /* a HIP runtime call failed */
    TT_E_BUDGET = -8,       /* the request does not fit the scratch budget */
    TT_E_TOO_LARGE = -9     /* n or m beyond the supported range */
};

/* Per-query counters (optional output of the _ex calls). */
typedef struct {
    uint64_t candidate_edges;     /* oriented edges that passed the bound test, all passes */
    uint64_t intersected_entries; /* adjacency entries read by intersections, all passes */
    uint64_t triangles_emitted;   /* triangles written to the candidate buffer */
    uint64_t edges_streamed;      /* oriented edges read by the filter, all passes */
    uint64_t distinct_sampled;    /* sampling only: distinct edges drawn */
    uint32_t passes;              /* enumeration passes (threshold bands and restarts) */
    uint32_t restarts;            /* passes repeated because the candidate buffer overflowed */
    double enum_ms;               /* device time from the first to the last enumeration pass */
    double select_ms;             /* device time of selection and output (HIP events) */
    double total_ms;              /* host wall time of the call */
    double enum_kernel_ms;        /* sum over passes of the enumeration kernel's own duration */
    double sample_ms;             /* sampling only: device time of the draws (and prefix sums) */
    uint64_t bound_order;         /* 1 if the passes streamed the entries in order of their bound
                                     for this p (built once this p has streamed > 4m entries) */
    uint64_t heavy_candidates;    /* candidates whose intersection was spread over many waves */
    uint64_t heavy_overflow;      /* heavy candidates beyond a pass's list, kept by their wave */
} tt_query_stats;

/*
 * Loads a graph from HOST arrays src[m], dst[m], w[m] (edge e = {src[e], dst[e]} with weight
 * w[e]).  Validation order: vertex range, self-loop, zero weight, duplicate pair (Sec. 1
 * requires a simple graph with positive weights); the first failing rule is reported.
 * Builds the degree-oriented CSR on the device (every triangle is reached exactly once from
 * its two lowest vertices in (degree, ID) order, the orientation of the brute-force
 * enumerator of Sec. 3).  *out receives the handle; free it with graph_free.
 */
int graph_load(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
               tt_graph **out);

/*
 * As graph_load, but src/dst/w are DEVICE pointers (e.g. from torch tensors) and all work is
 * ordered on `stream` (a hipStream_t; NULL = the default stream).  The graph keeps using that
 * stream for its queries.  The input buffers are read during the call only.
 */
int graph_load_device(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                      void *stream, tt_graph **out);

/*
 * Exact top-k triangles by m_p (Eq. 1).  out: caller-owned HOST array with room for k
 * records.  k = 0 returns TT_OK with *n_out = 0.  p may be any double (+-INFINITY allowed);
 * NaN gives TT_E_ARG.
 */
int topk_triangles(tt_graph *g, uint32_t k, double p, tt_triangle *out, uint32_t *n_out);

/*
 * topk_triangles restricted to triangles that touch `subset` (at least one vertex in it),
 * subset: HOST array of subset_n vertex IDs (duplicates allowed; subset_n = 0 or subset =
 * NULL means no restriction).  stats may be NULL.
 */
int topk_triangles_ex(tt_graph *g, uint32_t k, double p, const uint32_t *subset, uint32_t subset_n,
                      tt_triangle *out, uint32_t *n_out, tt_query_stats *stats);

/*
 * topk_triangles for callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  It computes exactly what topk_triangles computes
 * (same kernels) but allocates nothing: no device or pinned memory, no events, and nothing of
 * the graph built on first use (a weight-ordered stream or a bound order built by earlier
 * topk_triangles calls is used; otherwise the rows are streamed in row order).  Its device
 * scratch is one static array of 64 MiB per device, held by each device the library runs on
 * until the process ends, which keeps the last call's contents (each call clears what must
 * start at zero).  Calls on one device are serialised by a lock; the work runs on the graph's
 * stream and has finished when the call returns.  out: caller-owned HOST array of k records.
 * k > 16384 gives TT_E_TOO_LARGE.  No stats.
 */
int topk_triangles_noalloc(tt_graph *g, uint32_t k, double p, tt_triangle *out, uint32_t *n_out);

/*
 * Weighted edge sampling (Alg. 3): `budget` independent draws of an edge e with probability
 * w_e^q / Z (Prop. 1), q = p for finite p > 0 and q = 1 otherwise; the result is the top-k,
 * by the true m_p, of the union of all triangles on the drawn edges.  Draw s uses the s-th
 * output of SplitMix64 started from `seed` (Steele, Lea, Flood 2014) and selects the first
 * edge, in input order, whose inclusive prefix sum of w^q exceeds floor(x_s * Z / 2^64)
 * (integer q in {1, 2, 3}, exact 128-bit arithmetic) or (x_s >> 11) * 2^-53 * Z (other q, FP64).
 * budget = 0 or k = 0 returns TT_OK with *n_out = 0.
 */
int sample_heavy_triangles(tt_graph *g, uint32_t k, double p, uint64_t budget, uint64_t seed, tt_triangle *out,
                           uint32_t *n_out);

/*
 * sample_heavy_triangles with the sampling exponent named and the draws returned (Alg. 3;
 * Prop. 1 gives the probability of a triangle for any exponent).
 *   q      : edges are drawn with probability w_e^q / Z.  NaN selects the default reading
 *            above (q = p for finite p > 0, else 1); otherwise q must be finite and > 0, else
 *            TT_E_ARG.  The draw rule is the one above for this q (exact 128-bit for q in
 *            {1, 2, 3}, FP64 prefix sums otherwise).  Ranking always uses the true m_p.
 *   draws  : NULL, or a caller-owned HOST array of `budget` uint32 that receives the input
 *            edge index of every draw, in draw order (draw s at draws[s]).  With draws given,
 *            k = 0 runs the draws only.
 *   stats  : may be NULL.
 */
int sample_heavy_triangles_ex(tt_graph *g, uint32_t k, double p, uint64_t budget, uint64_t seed, double q,
                              uint32_t *draws, tt_triangle *out, uint32_t *n_out, tt_query_stats *stats);

/*
 * Weighted wedge sampling (Alg. 4) and weighted path sampling (Alg. 5): `budget` independent
 * draws of a wedge (scheme TT_SAMPLE_WEDGE: a centre a by Eq. wedgeone, b and c in N(a) by Eqs.
 * wedgetwo and wedgethree) or of a three-edge path (TT_SAMPLE_PATH: an edge (a, b) by Eq.
 * pathone, c in N(a) \ b and c' in N(b) \ a by Eqs. pathtwo and paththree), each with edge
 * weights raised to the sampling exponent q (NaN: q = p for finite p > 0, else 1).  A wedge
 * draw finds triangle {a, b, c} when b != c and {b, c} is an edge; a path draw when c' = c.  The
 * result is the top-k, by the true m_p, of the distinct triangles found (Props. 2 and 3 give
 * each triangle's probability per draw: proportional to the sum of its edges' w^q).  Draw s
 * uses the SplitMix64 outputs 3s, 3s+1, 3s+2 of `seed`; the sampling tables are FP64.
 *   draws : NULL, or a HOST array of 4 * budget uint32: per draw (a, b, c, x) with x = 1 if the
 *           wedge closed (else 0), or x = c' for a path.  With draws given, k = 0 draws only.
 *   stats : may be NULL.
 * Graphs of more than 2^21 vertices or with 2m >= 2^31 give TT_E_TOO_LARGE; budget <= 2^31.
 * The symmetric adjacency (rows sorted by neighbour) is built by the first call on a graph.
 */
enum { TT_SAMPLE_WEDGE = 1, TT_SAMPLE_PATH = 2 };
typedef struct {
    uint64_t closed_draws;       /* draws that found a triangle */
    uint64_t distinct_triangles; /* distinct triangles among them */
} tt_sampler_stats;
int sample_triangles_by(tt_graph *g, int scheme, uint32_t k, double p, uint64_t budget, uint64_t seed, double q,
                        uint32_t *draws, tt_triangle *out, uint32_t *n_out, tt_sampler_stats *stats);

/*
 * Weighted edge sampling extended to cliques (Sec. 4.5, Appendix A): `budget` edge draws as in
 * sample_heavy_triangles (exponent q, NaN for the default reading), then every clique of `size`
 * (4 or 5) vertices that contains a drawn edge; the result is the top-k of those cliques by the
 * generalized p-mean of their size (size - 1) / 2 edge weights (Eq. 1 over the clique's edges),
 * sorted by score descending, then by the sorted vertex IDs.  The order is exact for p in
 * {-inf, 1, +inf} (integer keys) and decided by the FP64 mean otherwise.  flags =
 * TT_CLIQUE_ALL_EDGES takes every edge instead of draws (the exact top-k cliques).  *found (may be
 * NULL) receives the number of distinct cliques on the drawn edges.  A drawn edge whose ends have
 * more than 512 common neighbours gives TT_E_TOO_LARGE (this sampler is meant for the small
 * graphs of the appendix).  Builds the symmetric adjacency on first use (2m < 2^31).
 */
typedef struct {
    uint32_t v[5];  /* vertex IDs ascending (v[4] = 0 for 4-cliques) */
    uint32_t size;  /* 4 or 5 */
    double score;   /* the generalized p-mean of the clique's edge weights */
} tt_clique;
enum { TT_CLIQUE_ALL_EDGES = 1 };
int sample_heavy_cliques(tt_graph *g, uint32_t size, uint32_t k, double p, uint64_t budget, uint64_t seed, double q,
                         uint32_t flags, tt_clique *out, uint32_t *n_out, uint64_t *found);

/*
 * Static heavy-light (Alg. 1, Sec. 3): the edges heavier than tau form H, and the answer is the
 * top-k, by m_p, of the triangles of the subgraph G[H] (all three edges heavier than tau) — an
 * approximation of the top-k of G that becomes exact as tau falls (tau = 0 keeps every edge).
 * out: HOST, room for k records.  *heavy_edges (may be NULL) receives |H|.  The graph is not
 * changed; G[H] is built on the device for the call and released after it.
 */
int shl_topk_triangles(tt_graph *g, uint32_t k, double p, uint32_t tau, tt_triangle *out, uint32_t *n_out,
                       uint64_t *heavy_edges);

/*
 * Serving: a request loop over one resident graph.  Callers: services that answer a stream of
 * top-k queries (any k, any p, optionally restricted to a vertex subset as in
 * topk_triangles_ex) on a graph kept in device memory.  Each of `slots` workers owns a HIP
 * stream and its query scratch, so admitted requests overlap on the device.  Requests wait in
 * FIFO order and are admitted when a worker is free and their scratch bytes
 * (server_request_bytes) fit into `scratch_budget` together with the requests already
 * running; a request arriving while others run is admitted as soon as one finishes.  A worker
 * keeps its scratch between requests (it grows with k), and that retained scratch is what the
 * budget bounds: a request is admitted on a free worker when the worker's scratch, grown to the
 * request's need, fits the budget together with the scratch every other worker holds.  Every
 * result is exactly the result of topk_triangles_ex for the same arguments.  The graph must
 * outlive the server and must not be freed while it runs.  All calls are thread-safe.
 */
typedef struct tt_server tt_server;

/* slots in [1, 64]; scratch_budget in bytes of device memory. */
int server_create(tt_graph *g, uint32_t slots, uint64_t scratch_budget, tt_server **out);

/* Device scratch bytes a request with this k and subset size is charged at admission. */
uint64_t server_request_bytes(tt_server *s, uint32_t k, uint32_t subset_n);

/* Queues a request; *ticket identifies it.  subset: HOST array copied before return.
 * TT_E_BUDGET if the request can never fit the budget; TT_E_VERTEX_RANGE for a bad subset. */
int server_submit(tt_server *s, uint32_t k, double p, const uint32_t *subset, uint32_t subset_n,
                  uint64_t *ticket);

/* *done = 1 once the request has finished (its result waits for server_wait).  TT_E_ARG (and
 * *done = 0) for a ticket that is not outstanding: never issued, or already released by
 * server_wait. */
int server_poll(tt_server *s, uint64_t ticket, int *done);

/* Blocks until the request has finished, then returns its result (out: HOST, room for k) and
 * releases the ticket.  stats->total_ms is the time from submission to completion.  TT_E_ARG for
 * a ticket that is not outstanding (never issued, or released by an earlier or concurrent
 * server_wait): it never blocks on such a ticket. */
int server_wait(tt_server *s, uint64_t ticket, tt_triangle *out, uint32_t *n_out, tt_query_stats *stats);

/* Device bytes the workers' scratch holds now (what the scratch budget bounds; lazily built graph
 * state belongs to the graph, graph_device_bytes). */
uint64_t server_scratch_bytes(tt_server *s);

/* Counters since creation: admitted and completed requests, peak charged scratch bytes,
 * longest queue and most requests running at once.  Any pointer may be NULL. */
int server_info(tt_server *s, uint64_t *admitted, uint64_t *completed, uint64_t *peak_bytes,
                uint32_t *max_queue, uint32_t *max_running);

/* Finishes every queued request, then stops the workers and frees their memory.  NULL-safe. */
void server_destroy(tt_server *s);

/*
 * Batched form: one top-k per graph for many independent graphs (the problem of Sec. 1 for
 * each of them), answered by one captured launch sequence.  The graphs are concatenated:
 * graph g has n[g] vertices with LOCAL ids 0..n[g]-1 and m[g] edges, stored at positions
 * eoff[g] .. eoff[g]+m[g]-1 of src/dst/w, eoff being the exclusive prefix sum of m.  Every
 * graph must be simple with positive weights (validated as in graph_load; a vertex id >= n[g]
 * gives TT_E_VERTEX_RANGE naming the graph).  Together the graphs may hold at most 2^32 - 2
 * vertices and 2^32 - 2 edges.  Inputs are copied; *out receives the handle.
 */
typedef struct tt_batch tt_batch;

/* n[count], m[count]: HOST arrays; src/dst/w: HOST arrays of sum(m) entries. */
int batch_load(uint32_t count, const uint32_t *n, const uint64_t *m, const uint32_t *src,
               const uint32_t *dst, const uint32_t *w, tt_batch **out);

/* As batch_load with src/dst/w in DEVICE memory (n and m stay on the host), read on `stream`
 * (a hipStream_t) in order with the work that produced them; with NULL the null stream is
 * synchronised first. */
int batch_load_device(uint32_t count, const uint32_t *n, const uint64_t *m, const uint32_t *src,
                      const uint32_t *dst, const uint32_t *w, void *stream, tt_batch **out);

/* Counters and launch choices of one batched query (optional output of batch_topk_ex). */
typedef struct {
    uint64_t candidate_edges, intersected_entries, triangles_emitted, edges_streamed;
    uint32_t config;           /* launch configuration used (index, see batch_topk_ex) */
    uint32_t growth;           /* rank ratio between consecutive score bands */
    uint32_t filter_blocks, intersect_blocks;
    uint32_t passes;           /* score bands captured (the last one exhaustive) */
    uint32_t restart_rounds;   /* overflow restart rounds captured after the selection */
    uint32_t restarts;         /* graphs redone because their triangle region overflowed */
    uint32_t merge_max;        /* intersection choice: rows with at most this many entries
                                  together are merged by one lane, longer ones binary-searched */
    double launch_ms;          /* device time of the captured sequence (HIP events) */
    double tune_ms;            /* host time spent by the autotuner in this call (first use) */
    double total_ms;           /* host wall time of the call */
} tt_batch_stats;

enum { TT_BATCH_EAGER = 1 }; /* run the launch sequence directly instead of its captured graph */

/*
 * out: HOST, count*k triangles; graph g's top min(k, T_g) are out[g*k ...] in local ids,
 * sorted as topk_triangles sorts them, the rest of its k slots zero; n_out: HOST, count
 * values.  config = -1 uses the
 * autotuner's choice for this (k, p) (launch shape, number of bands and of captured restart
 * rounds, timed on first use), or 0 .. batch_num_configs()-1 forces a launch shape with the
 * full number of bands.  Every choice and both launch modes return exactly the same result.
 * Calls on one batch are serialised.
 */
int batch_topk_ex(tt_batch *b, uint32_t k, double p, int config, uint32_t flags, tt_triangle *out,
                  uint32_t *n_out, tt_batch_stats *stats);
int batch_topk(tt_batch *b, uint32_t k, double p, tt_triangle *out, uint32_t *n_out);

/* Number of launch configurations the autotuner chooses from. */
uint32_t batch_num_configs(void);

/* Number of graphs (0 for NULL). */
uint32_t batch_num_graphs(const tt_batch *b);

/* Releases every resource of b.  NULL-safe. */
void batch_free(tt_batch *b);

/* Number of vertices / undirected edges of a loaded graph (0 for NULL). */
uint32_t graph_num_vertices(const tt_graph *g);
uint64_t graph_num_edges(const tt_graph *g);

/* Device bytes held by the graph (CSR, copies and cached scratch). */
uint64_t graph_device_bytes(const tt_graph *g);

/* Releases every resource of g.  NULL-safe.  Its device blocks go to a process-wide cache
 * (per device, up to 3/4 of that device's memory) that later loads, queries and batches reuse. */
void graph_free(tt_graph *g);

/* Returns every cached device block of every device to the driver; blocks in use by live graphs,
 * batches or servers are untouched.  Returns the bytes released.  Call it when other code in the
 * process (e.g. a tensor allocator) needs the memory.  Thread-safe; never fails. */
uint64_t tt_trim_cache(void);

/* Message for the last error on the calling thread ("" if none).  Valid until the next call. */
const char *tt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TOPKTRI_H */
