// scan.h — prefix sums used by the CSR build and by weighted edge sampling.
#pragma once
#include "common.h"

// Inclusive prefix sums of w_e^q over input edges e = 0..m-1 (weights in input order, in_w).
// q = 1: uint64_t[m]; q = 2 or 3: u128[m]; any other q: double[m].  With tmp (at least
// scan_tmp_bytes(m) bytes, kept by the caller until the stream has run the scan) nothing is
// allocated and the call does not wait; without it the call waits for the scan.
int inclusive_weight_prefix(tt_graph *g, double q, void *out, void *tmp = nullptr);

// Inclusive prefix sums of n doubles on stream s (tmp as above).
int inclusive_scan_f64(const double *in, double *out, uint64_t n, hipStream_t s, void *tmp = nullptr);
