/*
 * topktri_dhl.h — the paper's exact method on the CPU (libtopktri_dhl.so): the dynamic
 * heavy-light algorithm (Alg. 2, Sec. 3.1) and its distribution-oblivious variant Auto-HL
 * (Sec. 3.3), for the same problem as topktri.h (Sec. 1, Eq. 1) and with the same result
 * conventions (tt_triangle, order by score descending then (i, j, l) ascending, status codes).
 * It is a CPU program beside the GPU library, not a fallback of it: nothing in libtopktri.so
 * calls it.
 */
#ifndef TOPKTRI_DHL_H
#define TOPKTRI_DHL_H

#include <stdint.h>

#include "topktri.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Counters and phase times of one call. */
typedef struct {
    uint64_t enumerated; /* triangles enumerated (each exactly once) */
    uint64_t h_moves;    /* edges moved from heavy to super-heavy */
    uint64_t l_moves;    /* edges moved from light to heavy */
    uint64_t lookups;    /* adjacency entries scanned by the moves */
    uint64_t final_h;    /* super-heavy edges at the end */
    uint64_t final_l;    /* super-heavy and heavy edges at the end */
    double sort_ms;      /* sorting the edges by weight */
    double build_ms;     /* validation, sort and adjacency */
    double loop_ms;      /* the pointer loop and the output */
    double total_ms;
} tt_dhl_stats;

/*
 * Exact top-k triangles by m_p.  src, dst, w: HOST arrays of m edges (validated as graph_load
 * validates them: vertex range, self-loop, zero weight, duplicate pair).  alpha > 0 runs
 * Alg. 2 with pointer exponent alpha (the paper's experiments use 1.25 at p = 1); alpha = 0
 * runs Auto-HL.  threads: OpenMP threads for the sort and the adjacency build (0: all); the
 * pointer loop is sequential, as in the paper.  out: HOST, room for k records; *n_out =
 * min(k, T).  stats may be NULL.  Returns TT_OK or a TT_E_* code (dhl_last_error() describes
 * it).
 */
int dhl_topk_triangles(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst, const uint32_t *w,
                       uint32_t k, double p, double alpha, int threads, tt_triangle *out, uint32_t *n_out,
                       tt_dhl_stats *stats);

/* Message for the last error on the calling thread ("" if none). */
const char *dhl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TOPKTRI_DHL_H */
