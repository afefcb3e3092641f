/*
 * graphgen.c — seeded synthetic inputs for the top-k weighted triangle problem.
 *
 * This file produces INPUTS only: edge lists and edge weights. It contains none of
 * the method's arithmetic (no triangle enumeration, no p-mean, no selection), and
 * both the CPU oracle and the GPU library consume what it writes.
 *
 * Graph model.  The paper analyses a configuration model with power-law degrees and
 * power-law (heavy-tailed) edge weights (Sec. 3.3, "Analysis for power-law distributed
 * weights", and Fig. 1).  Its datasets are not available, so a Chung-Lu graph stands in
 * for them: vertex i gets expected degree t_i = c * (i+1)^(-1/(gamma-1)), capped at
 * sqrt(2m) so that every pair probability t_u t_v / S stays <= 1, with c chosen so that
 * sum(t) = 2m.  Each pair {u,v} is then present independently with probability
 * min(t_u t_v / S, 1).  The pairs are drawn with the skipping method of Miller and
 * Hagberg ("Efficient generation of networks with given expected degrees", WAW 2011),
 * which visits only O(n + m) candidates and never produces a duplicate or a self-loop.
 * Vertex labels are then permuted with a seeded Fisher-Yates shuffle so that IDs do not
 * correlate with degree.
 *
 * Weights are Zipf(s) truncated to {1, ..., wmax}: P(w = x) proportional to x^(-s),
 * drawn by inverse CDF from a per-edge counter-based uniform.
 *
 * Randomness is counter-based: every uniform is a hash of (seed, stream, index), so the
 * output does not depend on the number of threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

enum { GG_OK = 0, GG_E_ARG = -1, GG_E_NOMEM = -2, GG_E_CAPACITY = -3 };

enum {
    S_EDGE = 0x45444745ull,   /* "EDGE" */
    S_W = 0x57454947ull,      /* "WEIG" */
    S_PERM = 0x5045524dull,   /* "PERM" */
    S_PLANT = 0x504c414eull,  /* "PLAN" */
    S_PLANTW = 0x504c5757ull, /* "PLWW" */
};

/* 64-bit finaliser of SplitMix64 (Steele, Lea, Flood 2014). */
static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static inline uint64_t hash3(uint64_t seed, uint64_t stream, uint64_t idx) {
    uint64_t h = mix64(seed + 0x9E3779B97F4A7C15ull);
    h = mix64(h ^ (stream * 0xD1B54A32D192ED03ull));
    return mix64(h ^ (idx + 0x632BE59BD9B4E019ull));
}
/* uniform in the open interval (0, 1) */
static inline double u01(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

/* ---------------------------------------------------------------- expected degrees */

/* Fills t[0..n) with capped power-law expected degrees summing to 2m (descending). */
static int expected_degrees(uint64_t n, uint64_t m, double gamma, double *t) {
    if (n < 2 || m == 0 || !(gamma > 1.0)) return GG_E_ARG;
    const double alpha = 1.0 / (gamma - 1.0);
    const double cap = sqrt(2.0 * (double)m);
    /* suffix sums of (i+1)^-alpha in long double so that the bisection below is O(log n) */
    long double *suf = (long double *)malloc((n + 1) * sizeof(long double));
    if (!suf) return GG_E_NOMEM;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < n; i++) t[i] = pow((double)(i + 1), -alpha);
    suf[n] = 0.0L;
    for (uint64_t i = n; i-- > 0;) suf[i] = suf[i + 1] + (long double)t[i];
    const long double target = 2.0L * (long double)m;
    double lo = 0.0, hi = cap * pow((double)n, alpha) * 4.0 + 1.0;
    for (int it = 0; it < 200; it++) {
        double c = 0.5 * (lo + hi);
        /* the capped vertices form a prefix: c * t_i >= cap  <=>  i + 1 <= (c/cap)^(1/alpha) */
        double jf = pow(c / cap, 1.0 / alpha);
        uint64_t j = jf >= (double)n ? n : (uint64_t)jf;
        while (j < n && c * t[j] >= cap) j++;
        while (j > 0 && c * t[j - 1] < cap) j--;
        long double s = (long double)j * cap + (long double)c * suf[j];
        if (s < target) lo = c; else hi = c;
        if (hi - lo <= 1e-15 * hi) break;
    }
    const double c = 0.5 * (lo + hi);
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < n; i++) {
        double v = c * t[i];
        t[i] = v < cap ? v : cap;
    }
    free(suf);
    return GG_OK;
}

/* ---------------------------------------------------------------- Zipf weights */

typedef struct { double *cdf; uint32_t wmax; } zipf_t;

static int zipf_init(zipf_t *z, double s, uint32_t wmax) {
    if (wmax == 0 || !(s > 0.0)) return GG_E_ARG;
    z->wmax = wmax;
    z->cdf = (double *)malloc((size_t)wmax * sizeof(double));
    if (!z->cdf) return GG_E_NOMEM;
    long double acc = 0.0L;
    for (uint32_t x = 1; x <= wmax; x++) { acc += powl((long double)x, -(long double)s); z->cdf[x - 1] = (double)acc; }
    const double tot = (double)acc;
    for (uint32_t x = 0; x < wmax; x++) z->cdf[x] /= tot;
    z->cdf[wmax - 1] = 1.0;
    return GG_OK;
}
static inline uint32_t zipf_draw(const zipf_t *z, double u) {
    uint32_t lo = 0, hi = z->wmax - 1; /* first index with cdf >= u */
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (z->cdf[mid] >= u) hi = mid; else lo = mid + 1;
    }
    return lo + 1;
}

/* ---------------------------------------------------------------- Chung-Lu pairs */

typedef struct { uint32_t *u, *v; uint64_t len, cap; } ebuf_t;
static int ebuf_push(ebuf_t *b, uint32_t u, uint32_t v) {
    if (b->len == b->cap) {
        uint64_t nc = b->cap ? b->cap * 2 : 1024;
        uint32_t *nu = (uint32_t *)realloc(b->u, nc * sizeof(uint32_t));
        if (!nu) return GG_E_NOMEM;
        b->u = nu;
        uint32_t *nv = (uint32_t *)realloc(b->v, nc * sizeof(uint32_t));
        if (!nv) return GG_E_NOMEM;
        b->v = nv;
        b->cap = nc;
    }
    b->u[b->len] = u; b->v[b->len] = v; b->len++;
    return GG_OK;
}

/*
 * Generates a weighted Chung-Lu graph into caller-provided arrays of capacity `cap`.
 * src/dst receive permuted vertex IDs, w the Zipf weights.  *m_out is the edge count.
 */
int gg_chung_lu(uint64_t n, uint64_t m, double gamma, double zipf_s, uint32_t wmax, uint64_t seed,
                uint64_t cap, uint32_t *src, uint32_t *dst, uint32_t *w, uint64_t *m_out) {
    if (!src || !dst || !w || !m_out || n > 0xFFFFFFFFull) return GG_E_ARG;
    double *t = (double *)malloc(n * sizeof(double));
    if (!t) return GG_E_NOMEM;
    int rc = expected_degrees(n, m, gamma, t);
    if (rc) { free(t); return rc; }
    long double S_ld = 0.0L;
    for (uint64_t i = 0; i < n; i++) S_ld += t[i];
    const double S = (double)S_ld;

    /* rows are split into blocks of roughly equal expected work; blocks are concatenated in
       order, so the output is independent of the thread count */
    const int NB = 4096;
    uint64_t *bstart = (uint64_t *)malloc((NB + 1) * sizeof(uint64_t));
    ebuf_t *bufs = (ebuf_t *)calloc(NB, sizeof(ebuf_t));
    if (!bstart || !bufs) { free(t); free(bstart); free(bufs); return GG_E_NOMEM; }
    {
        long double acc = 0.0L, step = (S_ld + (long double)n) / NB;
        int b = 0;
        bstart[0] = 0;
        for (uint64_t i = 0; i < n && b < NB - 1; i++) {
            acc += t[i] + 1.0;
            if (acc >= step * (b + 1)) bstart[++b] = i + 1;
        }
        while (b < NB) bstart[++b] = n;
    }
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < NB; b++) {
        ebuf_t *B = &bufs[b];
        for (uint64_t u = bstart[b]; u < bstart[b + 1] && !fail; u++) {
            uint64_t v = u + 1, draw = 0;
            const uint64_t stream = S_EDGE | (u << 32); /* one stream per row */
            if (v >= n) break;
            double p = t[u] * t[v] / S;
            if (p > 1.0) p = 1.0;
            while (v < n && p > 0.0) {
                if (p < 1.0) {
                    double r = u01(hash3(seed, stream, draw++));
                    double skip = floor(log(r) / log1p(-p));
                    if (skip >= (double)(n - v)) break;
                    v += (uint64_t)skip;
                }
                if (v < n) {
                    double q = t[u] * t[v] / S;
                    if (q > 1.0) q = 1.0;
                    double r = u01(hash3(seed, stream, draw++));
                    if (r < q / p) {
                        if (ebuf_push(B, (uint32_t)u, (uint32_t)v)) { fail = 1; break; }
                    }
                    p = q;
                    v++;
                }
            }
        }
    }
    free(t);
    uint64_t total = 0;
    for (int b = 0; b < NB; b++) total += bufs[b].len;
    if (fail || total > cap) {
        for (int b = 0; b < NB; b++) { free(bufs[b].u); free(bufs[b].v); }
        free(bufs); free(bstart);
        return fail ? GG_E_NOMEM : GG_E_CAPACITY;
    }
    /* label permutation (sequential Fisher-Yates on its own stream) */
    uint32_t *perm = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!perm) { for (int b = 0; b < NB; b++) { free(bufs[b].u); free(bufs[b].v); } free(bufs); free(bstart); return GG_E_NOMEM; }
    for (uint64_t i = 0; i < n; i++) perm[i] = (uint32_t)i;
    for (uint64_t i = n - 1; i > 0; i--) {
        uint64_t j = (uint64_t)(u01(hash3(seed, S_PERM, i)) * (double)(i + 1));
        if (j > i) j = i;
        uint32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
    }
    uint64_t *off = (uint64_t *)malloc((NB + 1) * sizeof(uint64_t));
    off[0] = 0;
    for (int b = 0; b < NB; b++) off[b + 1] = off[b] + bufs[b].len;
    zipf_t z;
    rc = zipf_init(&z, zipf_s, wmax);
    if (rc) { free(perm); free(off); for (int b = 0; b < NB; b++) { free(bufs[b].u); free(bufs[b].v); } free(bufs); free(bstart); return rc; }
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < NB; b++) {
        for (uint64_t e = 0; e < bufs[b].len; e++) {
            uint64_t g = off[b] + e;
            src[g] = perm[bufs[b].u[e]];
            dst[g] = perm[bufs[b].v[e]];
            w[g] = zipf_draw(&z, u01(hash3(seed, S_W, g)));
        }
        free(bufs[b].u); free(bufs[b].v);
    }
    free(z.cdf); free(perm); free(off); free(bufs); free(bstart);
    *m_out = total;
    return GG_OK;
}

/*
 * Plants `nc` disjoint cliques of `cs` vertices each.  Existing edges inside a clique get
 * their weight multiplied by `mult`; missing ones are appended (at index *m_io onward) with a
 * fresh Zipf weight times `mult`.  The planted vertex sets are written to `members`
 * (nc*cs entries).  Capacity `cap` bounds the arrays.
 */
int gg_plant_cliques(uint64_t n, uint64_t *m_io, uint64_t cap, uint32_t *src, uint32_t *dst, uint32_t *w,
                     uint32_t nc, uint32_t cs, uint32_t mult, double zipf_s, uint32_t wmax, uint64_t seed,
                     uint32_t *members) {
    if (!m_io || !src || !dst || !w || !members || cs < 2 || (uint64_t)nc * cs > n) return GG_E_ARG;
    int32_t *cid = (int32_t *)malloc(n * sizeof(int32_t));
    if (!cid) return GG_E_NOMEM;
    memset(cid, 0xFF, n * sizeof(int32_t));
    /* distinct vertices by rejection on a counter stream */
    uint64_t draw = 0;
    for (uint32_t c = 0; c < nc; c++) {
        for (uint32_t s = 0; s < cs; s++) {
            uint32_t v;
            do { v = (uint32_t)(hash3(seed, S_PLANT, draw++) % n); } while (cid[v] >= 0);
            cid[v] = (int32_t)c;
            members[c * cs + s] = v;
        }
    }
    const uint64_t m0 = *m_io;
    const uint32_t npair = cs * (cs - 1) / 2;
    uint8_t *seen = (uint8_t *)calloc((size_t)nc * npair, 1);
    if (!seen) { free(cid); return GG_E_NOMEM; }
    for (uint64_t e = 0; e < m0; e++) {
        int32_t a = cid[src[e]], b = cid[dst[e]];
        if (a >= 0 && a == b) {
            uint64_t wv = (uint64_t)w[e] * mult;
            w[e] = wv > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)wv;
            /* mark the pair as present */
            uint32_t x = src[e], y = dst[e], ix = 0, iy = 0;
            for (uint32_t s = 0; s < cs; s++) { if (members[a * cs + s] == x) ix = s; if (members[a * cs + s] == y) iy = s; }
            if (ix > iy) { uint32_t tmp = ix; ix = iy; iy = tmp; }
            uint32_t pi = 0;
            for (uint32_t i = 0; i < ix; i++) pi += cs - 1 - i;
            pi += iy - ix - 1;
            seen[(size_t)a * npair + pi] = 1;
        }
    }
    zipf_t z;
    int rc = zipf_init(&z, zipf_s, wmax);
    if (rc) { free(cid); free(seen); return rc; }
    uint64_t m = m0;
    for (uint32_t c = 0; c < nc; c++) {
        uint32_t pi = 0;
        for (uint32_t i = 0; i < cs; i++)
            for (uint32_t j = i + 1; j < cs; j++, pi++) {
                if (seen[(size_t)c * npair + pi]) continue;
                if (m >= cap) { free(cid); free(seen); free(z.cdf); return GG_E_CAPACITY; }
                uint64_t wv = (uint64_t)zipf_draw(&z, u01(hash3(seed, S_PLANTW, (uint64_t)c * npair + pi))) * mult;
                src[m] = members[c * cs + i];
                dst[m] = members[c * cs + j];
                w[m] = wv > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)wv;
                m++;
            }
    }
    free(cid); free(seen); free(z.cdf);
    *m_io = m;
    return GG_OK;
}

/* Zipf weights alone (for tests of the weight model). */
int gg_zipf(uint64_t count, double zipf_s, uint32_t wmax, uint64_t seed, uint32_t *out) {
    zipf_t z;
    int rc = zipf_init(&z, zipf_s, wmax);
    if (rc) return rc;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < count; i++) out[i] = zipf_draw(&z, u01(hash3(seed, S_W, i)));
    free(z.cdf);
    return GG_OK;
}
