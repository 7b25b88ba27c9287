// The harmonic sum's neighbours in a search pipeline (gfx950):
//
//   * k_power: the power spectrum the sum runs on, from complex FFT bins, with
//     optional inter-binning (Sec. 2 names the step; the half-bin amplitude of
//     a rectangular-window DFT is estimated as (pi/4)(F_m - F_{m+1}), the
//     estimate the paper's citation introduced).  Integer bin m:
//     fl(fl(fl(re re) + fl(im im)) scale); half bin m + 1/2:
//     fl(fl(fl(dr dr) + fl(di di)) scale_h) with dr, di the rounded
//     differences and scale_h = fl32(scale fl32(pi^2 / 16)).  Inter-binned
//     output interleaves them: out[2m] = bin m, out[2m + 1] = half bin.
//   * k_peaks: peak clustering of the dense outputs: a candidate (snr >
//     threshold, at least one harmonic) is kept if no bin of its spectrum
//     within `radius` bins beats it (a larger SNR, or an equal one at a lower
//     bin); kept peaks are compacted like the sums' candidates.
//
// Both stream HBM once (the window reads of k_peaks are only for the few bins
// above the threshold and hit L1/L2).
#include "hs_internal.h"

namespace hs {
namespace {

template <bool INTERBIN>
__global__ __launch_bounds__(kBlock) void k_power(const float2 *__restrict__ F, int64_t n, float sc, float sch,
                                                  float *__restrict__ out) {
    for (int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x; m < n; m += (int64_t)gridDim.x * kBlock) {
        const float2 a = F[m];
        const float p = (a.x * a.x + a.y * a.y) * sc;
        if constexpr (INTERBIN) {
            if (m + 1 < n) {
                const float2 b = F[m + 1];
                const float dr = a.x - b.x, di = a.y - b.y;
                const float h = (dr * dr + di * di) * sch;
                out[2 * m] = p;
                out[2 * m + 1] = h;
            } else {
                out[2 * m] = p;
            }
        } else {
            out[m] = p;
        }
    }
}

constexpr int kPeakStage = 64;

// blockIdx.y = spectrum (or 0), bins of the spectrum strided over blockIdx.x.
__global__ __launch_bounds__(kBlock) void k_peaks(PeakArgs a) {
    __shared__ hs_candidate s_stage[kBlock / 64][kPeakStage];
    Stage st{s_stage[threadIdx.x >> 6], 0};
    const int sp = blockIdx.y;
    int64_t off = 0, len = a.n_bins;
    if (a.offsets) {
        off = a.offsets[sp];
        len = a.offsets[sp + 1] - off;
        if (len < 0) len = 0;
    }
    const float *snr = a.snr + off;
    const uint8_t *harm = a.harm + off;
    for (int64_t t = blockIdx.x; t * kBlock < len; t += gridDim.x) {
        const int64_t n = t * kBlock + threadIdx.x;
        bool keep = false;
        float v = 0.0f;
        int hv = 0;
        if (n < len) {
            v = snr[n];
            hv = harm[n];
            keep = v > a.thr && hv > 0;
            if (keep) {
                const int64_t lo = n - a.radius > 0 ? n - a.radius : 0;
                const int64_t hi = n + a.radius + 1 < len ? n + a.radius + 1 : len;
                for (int64_t j = lo; j < hi && keep; ++j) {
                    const float w = snr[j];
                    if (j != n && (w > v || (w == v && j < n))) keep = false;
                }
            }
        }
        hs_candidate rec;
        rec.spectrum = (uint32_t)sp;
        rec.bin = (uint32_t)n;
        rec.snr = v;
        rec.harm = (uint16_t)hv;
        rec.drift = (uint16_t)(keep && a.drift ? a.drift[off + n] : 0);
        stage_push<kPeakStage>(st, a.cand, a.cap, a.count, keep, rec);
    }
    stage_flush(st, a.cand, a.cap, a.count);
}

}  // namespace

hipError_t launch_power(const void *fft, int64_t n, bool interbin, float sc, float sch, float *out, hipStream_t st) {
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > kPlainBlocks) blocks = kPlainBlocks;
    if (blocks < 1) blocks = 1;
    if (interbin)
        hipLaunchKernelGGL(k_power<true>, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const float2 *)fft, n, sc, sch,
                           out);
    else
        hipLaunchKernelGGL(k_power<false>, dim3((unsigned)blocks), dim3(kBlock), 0, st, (const float2 *)fft, n, sc, sch,
                           out);
    return hipGetLastError();
}

hipError_t launch_peaks(const PeakArgs &a, int groups, int64_t max_len, hipStream_t st) {
    int64_t per = (max_len + kBlock - 1) / kBlock;
    const int64_t cap = (kPlainBlocks + groups - 1) / groups;
    if (per > cap) per = cap;
    if (per < 1) per = 1;
    hipLaunchKernelGGL(k_peaks, dim3((unsigned)per, (unsigned)groups), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace hs
