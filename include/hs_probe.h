/*
 * hs_probe.h -- measurement aid of the harmonic-sum library (libhs_probe.so),
 * not part of the sum itself: the ceiling of the greedy walk's memory access
 * pattern on the device, with its arithmetic reduced to what keeps the loads
 * live.
 *
 * The greedy sum (Sec. 3.3, Eq. (5), Algorithm 2) reads, for fundamental n at
 * harmonic k, the pair x[k n + d], x[k n + d + 1] and moves d up by one when
 * the second is larger.  A wave of 64 consecutive fundamentals therefore
 * gathers at stride k and touches about 2k cache lines of 128 bytes per
 * harmonic, so the walk is bound by cache-line traffic rather than by the
 * bytes it uses.  hsp_gather runs exactly that pattern for K = 32 harmonics
 * over a working set of (mask + 1) floats (positions wrap modulo the set), so
 * the set's size decides where the lines come from: a set of a few MB stays
 * in every XCD's L2, one of hundreds of MB is served from beyond the L2.
 *
 *   x       device floats, at least mask + 2 elements (positions mask and
 *           mask + 1 are both read), mask + 1 a power of two, 2 <= mask + 1 <= 2^28.
 *   n_fund  fundamentals 0..n_fund-1, 1 <= n_fund < 2^31, walked with a grid
 *           stride by `blocks` workgroups of 256 threads (blocks >= 1).
 *   out     device floats, [blocks * 256]: the per-thread sums (keeps the loads
 *           live; the values mean nothing).
 *   stream  hipStream_t of the current device (NULL = default).
 * Returns 0, or the hipError_t of the launch.  Stream-ordered, allocates
 * nothing.
 */
#ifndef HS_PROBE_H
#define HS_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int hsp_gather(const float *x, uint32_t mask, int64_t n_fund, int32_t blocks, float *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HS_PROBE_H */
