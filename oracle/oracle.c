/*
 * oracle.c — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for the top-k weighted triangle problem
 * of Kumar, Liu, Charikar and Benson, "Retrieving Top Weighted Triangles in Graphs"
 * (WSDM 2020).  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code with the GPU library.
 *
 * What it computes
 *   - Problem statement (Sec. 1): G = (V, E, w) simple, undirected, positive weights; the
 *     weight of triangle (i,j,l) is the generalized p-mean of its three edge weights
 *     (Eq. 1), with the limits p = 0 (geometric mean), p = +inf (max), p = -inf (min)
 *     named in Sec. 1.  The answer is the k heaviest triangles.
 *   - Ties (the paper gives no rule): order by score descending, then by the original
 *     vertex IDs (i, j, l) ascending, with i < j < l.
 *   - Fewer than k triangles: all of them are returned (Sec. 3.2 assumes at least k).
 *   - Enumeration: every triangle exactly once, as (i<j<l) in original IDs, by walking each
 *     edge (i,j) with i<j and intersecting the sorted neighbour lists of i and j above j.
 *   - Selection: one bounded heap of the k best per thread, then a full sort of the union
 *     of the heaps, the brute-force-with-a-heap scheme of Sec. 3 ("maintain a heap of the
 *     top-weighted triangles").  The result is by construction the first k of the total
 *     order above.
 *   - Weighted edge sampling (Alg. 3, Prop. 1): t independent draws of an edge with
 *     probability w_e^q / Z, by inverse CDF over the edges in input order (q = p for finite
 *     p > 0, else 1, unless the caller names q); the result
 *     set is the union over the draws of every triangle on the drawn edge, i.e. every
 *     triangle that has at least one drawn edge.  The uniform draws come from SplitMix64
 *     (Steele, Lea, Flood, OOPSLA 2014) so the GPU can replay the same sequence.
 *
 * Scoring.  For p in {-inf, 0, 1, 2, +inf} the order is decided by an exact integer key
 * (min, product, sum, sum of squares, max), a monotone transform of m_p.  For any other p
 * the key is the FP64 value of m_p, evaluated in long double as
 *     m = s * exp( log1p( (1/3) sum_x expm1(p * log(x/s)) ) / p ),
 * s = max weight for p > 0 and min weight for p < 0, which is Eq. 1 rewritten so that no
 * power overflows and small |p| loses no digits.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <stdio.h>
#include <omp.h>

typedef unsigned __int128 u128;

enum {
    O_OK = 0, O_E_ARG = -1, O_E_SELF_LOOP = -2, O_E_DUP_EDGE = -3, O_E_ZERO_WEIGHT = -4,
    O_E_VERTEX_RANGE = -5, O_E_NOMEM = -6
};
enum { MODE_MAX = 0, MODE_MIN = 1, MODE_SUM = 2, MODE_SUMSQ = 3, MODE_PROD = 4, MODE_GEN = 5 };
enum { FILTER_NONE = 0, FILTER_EDGE_MARK = 1, FILTER_VERTEX_MARK = 2 };

/* ------------------------------------------------------------------ scoring (Eq. 1) */

int orc_mode(double p) {
    if (isinf(p)) return p > 0 ? MODE_MAX : MODE_MIN;
    if (p == 1.0) return MODE_SUM;
    if (p == 2.0) return MODE_SUMSQ;
    if (p == 0.0) return MODE_PROD;
    return MODE_GEN;
}

static long double gen_mean(long double p, uint32_t a, uint32_t b, uint32_t c) {
    long double x[3] = {(long double)a, (long double)b, (long double)c};
    long double mx = x[0], mn = x[0];
    for (int t = 1; t < 3; t++) { if (x[t] > mx) mx = x[t]; if (x[t] < mn) mn = x[t]; }
    long double s = p > 0 ? mx : mn;
    long double acc = 0.0L;
    for (int t = 0; t < 3; t++) acc += expm1l(p * logl(x[t] / s));
    return s * expl(log1pl(acc / 3.0L) / p);
}

/* Exact order key (or FP64 bits for a generic p) and FP64 score of one triangle. */
static void score3(int mode, double p, uint32_t a, uint32_t b, uint32_t c, u128 *key, double *score) {
    switch (mode) {
    case MODE_MAX: { uint32_t v = a > b ? a : b; v = v > c ? v : c; *key = v; *score = (double)v; break; }
    case MODE_MIN: { uint32_t v = a < b ? a : b; v = v < c ? v : c; *key = v; *score = (double)v; break; }
    case MODE_SUM: { uint64_t s = (uint64_t)a + b + c; *key = s; *score = (double)s / 3.0; break; }
    case MODE_SUMSQ: {
        u128 s = (u128)a * a + (u128)b * b + (u128)c * c;
        *key = s;
        *score = (double)sqrtl((long double)s / 3.0L);
        break;
    }
    case MODE_PROD: {
        u128 s = (u128)a * b * c;
        *key = s;
        *score = (double)cbrtl((long double)s);
        break;
    }
    default: {
        double d = (double)gen_mean((long double)p, a, b, c);
        uint64_t bits;
        memcpy(&bits, &d, 8);
        *key = bits; /* positive doubles order like their bit patterns */
        *score = d;
        break;
    }
    }
}

double orc_score(double p, uint32_t a, uint32_t b, uint32_t c, uint64_t *key_hi, uint64_t *key_lo) {
    u128 k; double s;
    score3(orc_mode(p), p, a, b, c, &k, &s);
    if (key_hi) *key_hi = (uint64_t)(k >> 64);
    if (key_lo) *key_lo = (uint64_t)k;
    return s;
}

/* ------------------------------------------------------------------ graph */

typedef struct { uint32_t nbr, w; uint64_t eid; } ent_t;
typedef struct { uint64_t n, m; uint64_t *rp; ent_t *e; } adj_t;

static int cmp_ent(const void *x, const void *y) {
    const ent_t *a = (const ent_t *)x, *b = (const ent_t *)y;
    return a->nbr < b->nbr ? -1 : a->nbr > b->nbr ? 1 : 0;
}

/* Validation order: vertex range, self-loop, zero weight, duplicate pair. */
static int check_edges(uint64_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w) {
    int range = 0, loop = 0, zero = 0;
    for (uint64_t e = 0; e < m; e++) {
        if (src[e] >= n || dst[e] >= n) range = 1;
        else if (src[e] == dst[e]) loop = 1;
        if (w[e] == 0) zero = 1;
    }
    if (range) return O_E_VERTEX_RANGE;
    if (loop) return O_E_SELF_LOOP;
    if (zero) return O_E_ZERO_WEIGHT;
    return O_OK;
}

static void adj_free(adj_t *g) { free(g->rp); free(g->e); g->rp = NULL; g->e = NULL; }

/* Symmetric adjacency with rows sorted by neighbour ID; detects duplicate pairs. */
static int adj_build(uint64_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w, adj_t *g) {
    int rc = check_edges(n, m, src, dst, w);
    if (rc) return rc;
    g->n = n; g->m = m;
    g->rp = (uint64_t *)calloc(n + 1, sizeof(uint64_t));
    g->e = (ent_t *)malloc((2 * m + 1) * sizeof(ent_t));
    if (!g->rp || !g->e) { adj_free(g); return O_E_NOMEM; }
    const int progress = getenv("ORC_PROGRESS") != NULL;
    for (uint64_t e = 0; e < m; e++) { g->rp[src[e] + 1]++; g->rp[dst[e] + 1]++; }
    for (uint64_t v = 0; v < n; v++) g->rp[v + 1] += g->rp[v];
    if (progress) fprintf(stderr, "[oracle] adjacency: degrees counted\n");
    uint64_t *cur = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    if (!cur) { adj_free(g); return O_E_NOMEM; }
    memcpy(cur, g->rp, (n + 1) * sizeof(uint64_t));
    for (uint64_t e = 0; e < m; e++) {
        ent_t a = {dst[e], w[e], e}, b = {src[e], w[e], e};
        g->e[cur[src[e]]++] = a;
        g->e[cur[dst[e]]++] = b;
    }
    free(cur);
    if (progress) fprintf(stderr, "[oracle] adjacency: entries placed\n");
    int dup = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : dup)
    for (uint64_t v = 0; v < n; v++) {
        uint64_t lo = g->rp[v], hi = g->rp[v + 1];
        qsort(g->e + lo, hi - lo, sizeof(ent_t), cmp_ent);
        for (uint64_t t = lo + 1; t < hi; t++)
            if (g->e[t].nbr == g->e[t - 1].nbr) dup = 1;
    }
    if (dup) { adj_free(g); return O_E_DUP_EDGE; }
    return O_OK;
}

int orc_validate(uint64_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w) {
    if (m && (!src || !dst || !w)) return O_E_ARG;
    adj_t g = {0};
    int rc = adj_build(n, m, src, dst, w, &g);
    adj_free(&g);
    return rc;
}

/* First index in row [lo, hi) whose neighbour is > x. */
static uint64_t first_above(const ent_t *e, uint64_t lo, uint64_t hi, uint32_t x) {
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (e[mid].nbr > x) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/*
 * Calls visit(ctx, tid, i, j, l, w_ij, w_il, w_jl, e_ij, e_il, e_jl) once per triangle
 * i < j < l, in parallel over i.
 */
typedef void (*visit_fn)(void *, int, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, uint32_t,
                         uint64_t, uint64_t, uint64_t);

static void enumerate(const adj_t *g, visit_fn visit, void *ctx) {
    const ent_t *E = g->e;
#pragma omp parallel for schedule(dynamic, 64)
    for (uint64_t i = 0; i < g->n; i++) {
        const int tid = omp_get_thread_num();
        const uint64_t ilo = g->rp[i], ihi = g->rp[i + 1];
        for (uint64_t a = first_above(E, ilo, ihi, (uint32_t)i); a < ihi; a++) {
            const uint32_t j = E[a].nbr;
            /* N(i) above j, N(j) above j */
            uint64_t x = a + 1, y = first_above(E, g->rp[j], g->rp[j + 1], j);
            const uint64_t yhi = g->rp[j + 1];
            while (x < ihi && y < yhi) {
                if (E[x].nbr < E[y].nbr) x++;
                else if (E[x].nbr > E[y].nbr) y++;
                else {
                    visit(ctx, tid, (uint32_t)i, j, E[x].nbr, E[a].w, E[x].w, E[y].w, E[a].eid, E[x].eid, E[y].eid);
                    x++; y++;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ top-k with heaps */

typedef struct { u128 key; uint32_t i, j, l; double score; } rec_t;

/* 1 if a ranks before b: larger key first, then smaller (i, j, l). */
static inline int better(const rec_t *a, const rec_t *b) {
    if (a->key != b->key) return a->key > b->key;
    if (a->i != b->i) return a->i < b->i;
    if (a->j != b->j) return a->j < b->j;
    return a->l < b->l;
}
static int cmp_rec(const void *x, const void *y) {
    const rec_t *a = (const rec_t *)x, *b = (const rec_t *)y;
    return better(a, b) ? -1 : better(b, a) ? 1 : 0;
}

typedef struct { rec_t *h; uint64_t size; uint64_t count; char pad[40]; } heap_t;

/* heap root = the worst record kept */
static void heap_push(heap_t *H, uint64_t k, const rec_t *r) {
    rec_t *h = H->h;
    if (H->size < k) {
        uint64_t c = H->size++;
        h[c] = *r;
        while (c > 0) {
            uint64_t p = (c - 1) / 2;
            if (better(&h[p], &h[c])) { rec_t t = h[p]; h[p] = h[c]; h[c] = t; c = p; } else break;
        }
    } else if (better(r, &h[0])) {
        h[0] = *r;
        uint64_t c = 0;
        for (;;) {
            uint64_t l = 2 * c + 1, rr = l + 1, worst = c;
            if (l < k && better(&h[worst], &h[l])) worst = l;
            if (rr < k && better(&h[worst], &h[rr])) worst = rr;
            if (worst == c) break;
            rec_t t = h[c]; h[c] = h[worst]; h[worst] = t; c = worst;
        }
    }
}

typedef struct {
    int mode; double p; uint64_t k;
    heap_t *heaps;
    const uint8_t *emark, *vmark; /* NULL: no condition */
} topk_ctx;

static void visit_topk(void *vctx, int tid, uint32_t i, uint32_t j, uint32_t l, uint32_t wij, uint32_t wil,
                       uint32_t wjl, uint64_t eij, uint64_t eil, uint64_t ejl) {
    topk_ctx *c = (topk_ctx *)vctx;
    if (c->emark && !(c->emark[eij] | c->emark[eil] | c->emark[ejl])) return;
    if (c->vmark && !(c->vmark[i] | c->vmark[j] | c->vmark[l])) return;
    rec_t r;
    score3(c->mode, c->p, wij, wil, wjl, &r.key, &r.score);
    r.i = i; r.j = j; r.l = l;
    heap_t *H = &c->heaps[tid];
    H->count++;
    if (c->k) heap_push(H, c->k, &r);
}

/*
 * Top-k triangles by (score desc, i, j, l).  Writes min(k, T) records; *t_total = T (the
 * number of triangles admitted).  A triangle is admitted if emark is NULL or one of its
 * edges is marked (emark[] over input edge IDs), and vmark is NULL or one of its vertices is
 * marked (vmark[] over vertices).
 */
int orc_topk_marked(uint64_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                    uint64_t k, double p, int nthreads, const uint8_t *emark, const uint8_t *vmark, uint32_t *oi,
                    uint32_t *oj, uint32_t *ol, double *oscore, uint64_t *okey_hi, uint64_t *okey_lo,
                    uint64_t *n_out, uint64_t *t_total) {
    if (n_out) *n_out = 0;
    if (isnan(p) || (m && (!src || !dst || !w)) || !n_out) return O_E_ARG;
    if (k && (!oi || !oj || !ol || !oscore)) return O_E_ARG;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    adj_t g = {0};
    int rc = adj_build(n, m, src, dst, w, &g);
    if (rc) return rc;
    const int T = omp_get_max_threads();
    heap_t *heaps = (heap_t *)calloc(T, sizeof(heap_t));
    if (!heaps) { adj_free(&g); return O_E_NOMEM; }
    for (int t = 0; t < T; t++) {
        heaps[t].h = (rec_t *)malloc((k ? k : 1) * sizeof(rec_t));
        if (!heaps[t].h) { for (int u = 0; u < T; u++) free(heaps[u].h); free(heaps); adj_free(&g); return O_E_NOMEM; }
    }
    topk_ctx ctx = {orc_mode(p), p, k, heaps, emark, vmark};
    enumerate(&g, visit_topk, &ctx);
    uint64_t total = 0, kept = 0;
    for (int t = 0; t < T; t++) { total += heaps[t].count; kept += heaps[t].size; }
    rec_t *all = (rec_t *)malloc((kept ? kept : 1) * sizeof(rec_t));
    if (!all) { for (int u = 0; u < T; u++) free(heaps[u].h); free(heaps); adj_free(&g); return O_E_NOMEM; }
    uint64_t pos = 0;
    for (int t = 0; t < T; t++) { memcpy(all + pos, heaps[t].h, heaps[t].size * sizeof(rec_t)); pos += heaps[t].size; }
    qsort(all, kept, sizeof(rec_t), cmp_rec);
    uint64_t out = kept < k ? kept : k;
    for (uint64_t r = 0; r < out; r++) {
        oi[r] = all[r].i; oj[r] = all[r].j; ol[r] = all[r].l; oscore[r] = all[r].score;
        if (okey_hi) okey_hi[r] = (uint64_t)(all[r].key >> 64);
        if (okey_lo) okey_lo[r] = (uint64_t)all[r].key;
    }
    *n_out = out;
    if (t_total) *t_total = total;
    free(all);
    for (int t = 0; t < T; t++) free(heaps[t].h);
    free(heaps);
    adj_free(&g);
    return O_OK;
}

/*
 * The triangles that contain a marked edge, found from the marked edges themselves: for each
 * marked edge {a, b}, every c in N(a) and N(b) (a merge of the two rows), reported once, from
 * the marked edge of smallest input ID among its edges.  The same set as enumerate() followed
 * by the edge-mark filter, at a cost that follows the marked edges' degrees instead of the
 * whole graph's triangles (the union of Alg. 3, step by step).  With ORC_PROGRESS set in the
 * environment, a line per tenth of the marked edges goes to stderr.
 */
static void enumerate_on_marked(const adj_t *g, const uint32_t *src, const uint32_t *dst, const uint8_t *emark,
                                visit_fn visit, void *ctx) {
    const ent_t *E = g->e;
    const int progress = getenv("ORC_PROGRESS") != NULL;
    uint64_t next = g->m / 10 + 1;
#pragma omp parallel for schedule(dynamic, 256)
    for (uint64_t e = 0; e < g->m; e++) {
        if (progress && omp_get_thread_num() == 0 && e >= next) {
            fprintf(stderr, "[oracle] marked-edge enumeration: edge %llu of %llu\n", (unsigned long long)e,
                    (unsigned long long)g->m);
            next += g->m / 10 + 1;
        }
        if (!emark[e]) continue;
        const uint32_t a = src[e], b = dst[e];
        uint64_t x = g->rp[a], y = g->rp[b];
        const uint64_t xe = g->rp[a + 1], ye = g->rp[b + 1];
        uint32_t wab = 0;
        while (x < xe && y < ye) {
            if (E[x].nbr < E[y].nbr) x++;
            else if (E[x].nbr > E[y].nbr) y++;
            else {
                const uint32_t c = E[x].nbr;
                const uint64_t eac = E[x].eid, ebc = E[y].eid;
                /* reported from its marked edge of smallest ID */
                if (!((emark[eac] && eac < e) || (emark[ebc] && ebc < e))) {
                    if (!wab) {
                        /* the weight of {a, b}: its entry in a's row */
                        uint64_t lo = g->rp[a], hi = xe;
                        while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (E[mid].nbr < b) lo = mid + 1; else hi = mid; }
                        wab = E[lo].w;
                    }
                    const uint32_t wac = E[x].w, wbc = E[y].w;
                    uint32_t v[3] = {a, b, c}, t;
                    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
                    if (v[1] > v[2]) { t = v[1]; v[1] = v[2]; v[2] = t; }
                    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
                    /* a pair holding a and b is {a, b}; else one holding a is {a, c}; else {b, c} */
#define PAIR_W(s0, s1) ((((s0) == a || (s1) == a) && ((s0) == b || (s1) == b)) ? wab : ((s0) == a || (s1) == a) ? wac : wbc)
#define PAIR_E(s0, s1) ((((s0) == a || (s1) == a) && ((s0) == b || (s1) == b)) ? e : ((s0) == a || (s1) == a) ? eac : ebc)
                    visit(ctx, omp_get_thread_num(), v[0], v[1], v[2], PAIR_W(v[0], v[1]), PAIR_W(v[0], v[2]),
                          PAIR_W(v[1], v[2]), PAIR_E(v[0], v[1]), PAIR_E(v[0], v[2]), PAIR_E(v[1], v[2]));
#undef PAIR_W
#undef PAIR_E
                }
                x++; y++;
            }
        }
    }
}

/*
 * Top-k of the triangles with a marked edge (emark[] over input edge IDs, required), and with
 * vmark given also a marked vertex: the result of orc_topk_marked with the same marks, found by
 * enumerate_on_marked.
 */
int orc_topk_on_marked_edges(uint64_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                             uint64_t k, double p, int nthreads, const uint8_t *emark, const uint8_t *vmark,
                             uint32_t *oi, uint32_t *oj, uint32_t *ol, double *oscore, uint64_t *okey_hi,
                             uint64_t *okey_lo, uint64_t *n_out, uint64_t *t_total) {
    if (n_out) *n_out = 0;
    if (isnan(p) || (m && (!src || !dst || !w || !emark)) || !n_out) return O_E_ARG;
    if (k && (!oi || !oj || !ol || !oscore)) return O_E_ARG;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    adj_t g = {0};
    int rc = adj_build(n, m, src, dst, w, &g);
    if (rc) return rc;
    if (getenv("ORC_PROGRESS")) fprintf(stderr, "[oracle] adjacency of %llu edges built\n", (unsigned long long)m);
    const int T = omp_get_max_threads();
    heap_t *heaps = (heap_t *)calloc(T, sizeof(heap_t));
    if (!heaps) { adj_free(&g); return O_E_NOMEM; }
    for (int t = 0; t < T; t++) {
        heaps[t].h = (rec_t *)malloc((k ? k : 1) * sizeof(rec_t));
        if (!heaps[t].h) { for (int u = 0; u < T; u++) free(heaps[u].h); free(heaps); adj_free(&g); return O_E_NOMEM; }
    }
    topk_ctx ctx = {orc_mode(p), p, k, heaps, NULL, vmark};
    enumerate_on_marked(&g, src, dst, emark, visit_topk, &ctx);
    uint64_t total = 0, kept = 0;
    for (int t = 0; t < T; t++) { total += heaps[t].count; kept += heaps[t].size; }
    rec_t *all = (rec_t *)malloc((kept ? kept : 1) * sizeof(rec_t));
    if (!all) { for (int u = 0; u < T; u++) free(heaps[u].h); free(heaps); adj_free(&g); return O_E_NOMEM; }
    uint64_t pos = 0;
    for (int t = 0; t < T; t++) { memcpy(all + pos, heaps[t].h, heaps[t].size * sizeof(rec_t)); pos += heaps[t].size; }
    qsort(all, kept, sizeof(rec_t), cmp_rec);
    uint64_t out = kept < k ? kept : k;
    for (uint64_t r = 0; r < out; r++) {
        oi[r] = all[r].i; oj[r] = all[r].j; ol[r] = all[r].l; oscore[r] = all[r].score;
        if (okey_hi) okey_hi[r] = (uint64_t)(all[r].key >> 64);
        if (okey_lo) okey_lo[r] = (uint64_t)all[r].key;
    }
    *n_out = out;
    if (t_total) *t_total = total;
    free(all);
    for (int t = 0; t < T; t++) free(heaps[t].h);
    free(heaps);
    adj_free(&g);
    return O_OK;
}

/* One filter: 0 none; 1 mark[] over input edge IDs; 2 mark[] over vertices. */
int orc_topk(uint64_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w, uint64_t k,
             double p, int nthreads, int filter, const uint8_t *mark, uint32_t *oi, uint32_t *oj, uint32_t *ol,
             double *oscore, uint64_t *okey_hi, uint64_t *okey_lo, uint64_t *n_out, uint64_t *t_total) {
    if (n_out) *n_out = 0;
    if ((filter && !mark) || filter < 0 || filter > FILTER_VERTEX_MARK) return O_E_ARG;
    return orc_topk_marked(n, m, src, dst, w, k, p, nthreads, filter == FILTER_EDGE_MARK ? mark : NULL,
                           filter == FILTER_VERTEX_MARK ? mark : NULL, oi, oj, ol, oscore, okey_hi, okey_lo,
                           n_out, t_total);
}

/* ------------------------------------------------------------------ cliques (Sec. 4.5) */

/* A clique of s vertices (ascending) and its order key / FP64 score. */
typedef struct { u128 key; uint32_t v[5]; double score; } clq_t;

static int clq_better(const clq_t *a, const clq_t *b, int s) {
    if (a->key != b->key) return a->key > b->key;
    for (int t = 0; t < s; t++)
        if (a->v[t] != b->v[t]) return a->v[t] < b->v[t];
    return 0;
}
static int clq_size_for_sort;
static int cmp_clq(const void *x, const void *y) {
    const clq_t *a = (const clq_t *)x, *b = (const clq_t *)y;
    return clq_better(a, b, clq_size_for_sort) ? -1 : clq_better(b, a, clq_size_for_sort) ? 1 : 0;
}

/* The generalized p-mean of E weights (Eq. 1 over a clique's edges): exact keys for p in
 * {-inf, 1, +inf} (min, sum, max), the FP64 value of the mean (long double evaluation) otherwise;
 * p = 0 is the geometric mean. */
static void clq_score(double p, const uint32_t *w, int E, u128 *key, double *score) {
    if (isinf(p)) {
        uint32_t r = w[0];
        for (int t = 1; t < E; t++) r = p > 0 ? (w[t] > r ? w[t] : r) : (w[t] < r ? w[t] : r);
        *key = r; *score = (double)r; return;
    }
    if (p == 1.0) {
        uint64_t r = 0;
        for (int t = 0; t < E; t++) r += w[t];
        *key = r; *score = (double)r / (double)E; return;
    }
    long double m;
    if (p == 0.0) {
        long double acc = 0.0L;
        for (int t = 0; t < E; t++) acc += logl((long double)w[t]);
        m = expl(acc / (long double)E);
    } else {
        long double sref = w[0];
        for (int t = 1; t < E; t++) { long double x = w[t]; if (p > 0 ? x > sref : x < sref) sref = x; }
        long double acc = 0.0L;
        for (int t = 0; t < E; t++) acc += expm1l((long double)p * logl((long double)w[t] / sref));
        m = sref * expl(log1pl(acc / (long double)E) / (long double)p);
    }
    double d = (double)m;
    uint64_t bits;
    memcpy(&bits, &d, 8);
    *key = bits; *score = d;
}

/* weight and edge ID of {x, y}, or 0 if not an edge */
static uint32_t adj_find(const adj_t *g, uint32_t x, uint32_t y, uint64_t *eid) {
    uint64_t lo = g->rp[x], hi = g->rp[x + 1];
    while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (g->e[mid].nbr < y) lo = mid + 1; else hi = mid; }
    if (lo < g->rp[x + 1] && g->e[lo].nbr == y) { *eid = g->e[lo].eid; return g->e[lo].w; }
    return 0;
}

/*
 * Top-k cliques of s = 4 or 5 vertices by the p-mean of their s (s - 1) / 2 edge weights,
 * ordered by score descending then the ascending vertex IDs; with emark, only cliques holding a
 * marked edge (input edge IDs).  Every clique is listed once, as i < j < x < y (< z), from the
 * common neighbours of i and j above j.  Writes min(k, T) cliques: ov[k * 5] (unused IDs 0),
 * oscore[k]; *t_total = T.
 */
int orc_cliques(uint64_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w, int s,
                uint64_t k, double p, int nthreads, const uint8_t *emark, uint32_t *ov, double *oscore,
                uint64_t *n_out, uint64_t *t_total) {
    if (n_out) *n_out = 0;
    if ((s != 4 && s != 5) || isnan(p) || (m && (!src || !dst || !w)) || !n_out || (k && (!ov || !oscore)))
        return O_E_ARG;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    adj_t g = {0};
    int rc = adj_build(n, m, src, dst, w, &g);
    if (rc) return rc;
    const int T = omp_get_max_threads();
    clq_t **lists = (clq_t **)calloc(T, sizeof(clq_t *));
    uint64_t *cnt = (uint64_t *)calloc(T, sizeof(uint64_t)), *cap = (uint64_t *)calloc(T, sizeof(uint64_t));
    if (!lists || !cnt || !cap) { free(lists); free(cnt); free(cap); adj_free(&g); return O_E_NOMEM; }
    int nomem = 0;
    const int E = s * (s - 1) / 2;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : nomem)
    for (uint64_t i = 0; i < n; i++) {
        const int tid = omp_get_thread_num();
        const ent_t *Ei = g.e;
        uint32_t *C = NULL;
        for (uint64_t a = first_above(Ei, g.rp[i], g.rp[i + 1], (uint32_t)i); a < g.rp[i + 1]; a++) {
            const uint32_t j = Ei[a].nbr;
            /* common neighbours of i and j above j */
            uint64_t x = a + 1, y = first_above(Ei, g.rp[j], g.rp[j + 1], j), nc = 0;
            const uint64_t xe = g.rp[i + 1], ye = g.rp[j + 1];
            free(C);
            C = (uint32_t *)malloc((xe - x + 1) * sizeof(uint32_t));
            if (!C) { nomem = 1; break; }
            while (x < xe && y < ye) {
                if (Ei[x].nbr < Ei[y].nbr) x++;
                else if (Ei[x].nbr > Ei[y].nbr) y++;
                else { C[nc++] = Ei[x].nbr; x++; y++; }
            }
            for (uint64_t p1 = 0; p1 < nc; p1++)
                for (uint64_t p2 = p1 + 1; p2 < nc; p2++) {
                    uint32_t V[5] = {(uint32_t)i, j, C[p1], C[p2], 0};
                    uint64_t e12;
                    if (!adj_find(&g, C[p1], C[p2], &e12)) continue;
                    /* a fifth vertex from the common neighbours after the fourth (5-cliques), or none */
                    const uint64_t z_lo = s == 5 ? p2 + 1 : 0, z_hi = s == 5 ? nc : 1;
                    for (uint64_t p3 = z_lo; p3 < z_hi; p3++) {
                        if (s == 5) V[4] = C[p3];
                        uint32_t W[10];
                        int marked = emark == NULL, e = 0, ok = 1;
                        for (int u = 0; u < s && ok; u++)
                            for (int v = u + 1; v < s; v++) {
                                uint64_t id;
                                uint32_t wt = adj_find(&g, V[u], V[v], &id);
                                if (!wt) { ok = 0; break; }
                                W[e++] = wt;
                                if (emark && emark[id]) marked = 1;
                            }
                        if (ok && marked) {
                            if (cnt[tid] == cap[tid]) {
                                uint64_t nc2 = cap[tid] ? 2 * cap[tid] : 1024;
                                clq_t *nl = (clq_t *)realloc(lists[tid], nc2 * sizeof(clq_t));
                                if (!nl) { nomem = 1; break; }
                                lists[tid] = nl;
                                cap[tid] = nc2;
                            }
                            clq_t *r = &lists[tid][cnt[tid]++];
                            memset(r, 0, sizeof(*r));
                            for (int u = 0; u < s; u++) r->v[u] = V[u];
                            clq_score(p, W, E, &r->key, &r->score);
                        }
                    }
                }
        }
        free(C);
    }
    uint64_t total = 0;
    for (int t = 0; t < T; t++) total += cnt[t];
    clq_t *all = nomem ? NULL : (clq_t *)malloc((total ? total : 1) * sizeof(clq_t));
    if (!all) {
        for (int t = 0; t < T; t++) free(lists[t]);
        free(lists); free(cnt); free(cap); adj_free(&g);
        return O_E_NOMEM;
    }
    uint64_t pos = 0;
    for (int t = 0; t < T; t++) { memcpy(all + pos, lists[t], cnt[t] * sizeof(clq_t)); pos += cnt[t]; free(lists[t]); }
    clq_size_for_sort = s;
    qsort(all, total, sizeof(clq_t), cmp_clq);
    const uint64_t out = total < k ? total : k;
    for (uint64_t r = 0; r < out; r++) {
        for (int u = 0; u < 5; u++) ov[r * 5 + u] = u < s ? all[r].v[u] : 0;
        oscore[r] = all[r].score;
    }
    *n_out = out;
    if (t_total) *t_total = total;
    free(all); free(lists); free(cnt); free(cap);
    adj_free(&g);
    return O_OK;
}

/* ------------------------------------------------------------------ listing (small graphs) */

typedef struct { uint32_t *i, *j, *l, *w3; uint64_t cap, cnt; } list_ctx;

static void visit_list(void *vctx, int tid, uint32_t i, uint32_t j, uint32_t l, uint32_t wij, uint32_t wil,
                       uint32_t wjl, uint64_t eij, uint64_t eil, uint64_t ejl) {
    (void)tid; (void)eij; (void)eil; (void)ejl;
    list_ctx *c = (list_ctx *)vctx;
    uint64_t pos;
#pragma omp atomic capture
    pos = c->cnt++;
    if (pos < c->cap) {
        c->i[pos] = i; c->j[pos] = j; c->l[pos] = l;
        c->w3[3 * pos] = wij; c->w3[3 * pos + 1] = wil; c->w3[3 * pos + 2] = wjl;
    }
}

/* Every triangle (unordered), with its weights (w_ij, w_il, w_jl).  *cnt = T. */
int orc_list(uint64_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w, uint64_t cap,
             uint32_t *oi, uint32_t *oj, uint32_t *ol, uint32_t *ow3, uint64_t *cnt) {
    if (!cnt || (m && (!src || !dst || !w)) || (cap && (!oi || !oj || !ol || !ow3))) return O_E_ARG;
    adj_t g = {0};
    int rc = adj_build(n, m, src, dst, w, &g);
    if (rc) return rc;
    list_ctx c = {oi, oj, ol, ow3, cap, 0};
    enumerate(&g, visit_list, &c);
    *cnt = c.cnt;
    adj_free(&g);
    return O_OK;
}

/* ------------------------------------------------------------------ weighted edge sampling */

/* i-th output (0-based) of SplitMix64 started from state `seed`. */
static inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Sampling exponent: q = p for finite p > 0, else 1. */
double orc_sample_exponent(double p) { return (isfinite(p) && p > 0.0) ? p : 1.0; }

/*
 * Alg. 3's draws: `budget` iid edges with P(e) = w_e^q / Z, by inverse CDF over the input
 * order.  Integer q in {1, 2, 3}: exact 128-bit prefix sums and r = floor(x * Z / 2^64) for
 * the 64-bit uniform x, so e = first index with prefix > r.  Other q: FP64 prefix sums in
 * input order and r = (x >> 11) * 2^-53 * Z.  Sets mark[e] = 1 for every drawn edge and,
 * if out_eids is not NULL, writes the draws in order.
 */
int orc_es_draw_q(uint64_t m, const uint32_t *w, double q, uint64_t budget, uint64_t seed, uint8_t *mark,
                  uint64_t *out_eids) {
    if (!mark || (m && !w) || !(q > 0.0) || isinf(q)) return O_E_ARG;
    if (m == 0 || budget == 0) return O_OK;
    const int exact = (q == 1.0 || q == 2.0 || q == 3.0);
    if (exact) {
        const int qi = (int)q;
        u128 *P = (u128 *)malloc(m * sizeof(u128));
        if (!P) return O_E_NOMEM;
        u128 acc = 0;
        for (uint64_t e = 0; e < m; e++) {
            u128 t = w[e];
            if (qi >= 2) t *= w[e];
            if (qi >= 3) t *= w[e];
            acc += t;
            P[e] = acc;
        }
        const u128 Z = acc;
        const uint64_t Zh = (uint64_t)(Z >> 64), Zl = (uint64_t)Z;
#pragma omp parallel for schedule(static)
        for (uint64_t s = 0; s < budget; s++) {
            const uint64_t x = splitmix64_at(seed, s);
            const u128 r = (u128)x * Zh + (uint64_t)(((u128)x * Zl) >> 64);
            uint64_t lo = 0, hi = m - 1;
            while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (P[mid] > r) hi = mid; else lo = mid + 1; }
            mark[lo] = 1;
            if (out_eids) out_eids[s] = lo;
        }
        free(P);
    } else {
        double *P = (double *)malloc(m * sizeof(double));
        if (!P) return O_E_NOMEM;
        double acc = 0.0;
        for (uint64_t e = 0; e < m; e++) { acc += pow((double)w[e], q); P[e] = acc; }
        const double Z = acc;
#pragma omp parallel for schedule(static)
        for (uint64_t s = 0; s < budget; s++) {
            const uint64_t x = splitmix64_at(seed, s);
            const double r = (double)(x >> 11) * (1.0 / 9007199254740992.0) * Z;
            uint64_t lo = 0, hi = m - 1;
            while (lo < hi) { uint64_t mid = lo + (hi - lo) / 2; if (P[mid] > r) hi = mid; else lo = mid + 1; }
            mark[lo] = 1;
            if (out_eids) out_eids[s] = lo;
        }
        free(P);
    }
    return O_OK;
}

/* The draws with the sampling exponent of p (q = p for finite p > 0, else 1). */
int orc_es_draw(uint64_t m, const uint32_t *w, double p, uint64_t budget, uint64_t seed, uint8_t *mark,
                uint64_t *out_eids) {
    if (isnan(p)) return O_E_ARG;
    return orc_es_draw_q(m, w, orc_sample_exponent(p), budget, seed, mark, out_eids);
}

/* The FP64 inclusive prefix sums of w^q in input order that the draws of a non-integer q
 * search (the same sequential sum as orc_es_draw_q). */
int orc_es_prefix_f64(uint64_t m, const uint32_t *w, double q, double *P) {
    if ((m && (!w || !P)) || !(q > 0.0) || isinf(q)) return O_E_ARG;
    double acc = 0.0;
    for (uint64_t e = 0; e < m; e++) { acc += pow((double)w[e], q); P[e] = acc; }
    return O_OK;
}

uint64_t orc_splitmix64_at(uint64_t seed, uint64_t i) { return splitmix64_at(seed, i); }
