// Host build of the library's scoring and pruning-bound functions (csrc/enum.h), for the CPU
// property tests in test_bounds.py.  Test infrastructure: nothing here runs on a GPU.
#include "../paper_1910_00692_amd/csrc/enum.h"

namespace {
Band make(int mode, double p, uint64_t Lhi, uint64_t Llo) {
    Band B{};
    B.L = ((u128)Lhi << 64) | Llo;
    B.Li = B.Lj = B.Ll = ~0u;
    B.mode = mode;
    B.p = p;
    B.theta = mode == MODE_GEN ? key_as_double(B.L) : 0.0;
    return B;
}
} // namespace

extern "C" {
int bt_mode(double p) { return mode_of(p); }
void bt_key(double p, uint32_t a, uint32_t b, uint32_t c, uint64_t *hi, uint64_t *lo) {
    const u128 k = score_key(mode_of(p), p, a, b, c);
    *hi = (uint64_t)(k >> 64);
    *lo = (uint64_t)k;
}
double bt_score(double p, uint64_t hi, uint64_t lo) { return key_to_score(mode_of(p), ((u128)hi << 64) | lo); }
int bt_bound_ok(double p, uint64_t Lhi, uint64_t Llo, uint32_t a, uint32_t Wu, uint32_t Wv) {
    const Band B = make(mode_of(p), p, Lhi, Llo);
    return B.mode == MODE_GEN ? bound_ok<true>(B, a, Wu, Wv) : bound_ok<false>(B, a, Wu, Wv);
}
uint64_t bt_min_other(double p, uint64_t Lhi, uint64_t Llo, uint32_t a, uint32_t W) {
    const Band B = make(mode_of(p), p, Lhi, Llo);
    return B.mode == MODE_GEN ? min_other<true>(B, a, W) : min_other<false>(B, a, W);
}
uint64_t bt_weight_floor(double p, uint64_t Lhi, uint64_t Llo, uint32_t W) {
    return weight_floor(mode_of(p), p, ((u128)Lhi << 64) | Llo, W);
}
uint64_t bt_score_floor(double p, uint64_t Lhi, uint64_t Llo) { return score_floor(mode_of(p), ((u128)Lhi << 64) | Llo); }
uint32_t bt_entry_bound(double p, uint32_t a, uint32_t Wu, uint32_t Wv) { return entry_bound(mode_of(p), p, a, Wu, Wv); }
uint32_t bt_weight_bin(uint32_t w) { return weight_bin(w); }
}
