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
// Both stream HBM once (k_peaks stages each tile's window in LDS, so the
// candidates' window checks are LDS reads).
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
constexpr int kPeakPer = 4;                        // bins per thread and tile (independent loads in flight)
constexpr int kPeakTile = kBlock * kPeakPer;
constexpr int kPeakLdsRadius = 1024;               // radii up to this read the window from LDS

// blockIdx.y = spectrum (or 0), tiles of kPeakTile bins of the spectrum
// strided over blockIdx.x; thread i owns bins t0 + i + kBlock j.  LDS: each
// tile's snr plus `radius` bins on either side (clamped to the spectrum), so
// the window checks of the candidates are LDS reads; larger radii read the
// window from global memory.
template <bool LDS>
__global__ __launch_bounds__(kBlock) void k_peaks(PeakArgs a) {
    __shared__ hs_candidate s_stage[kBlock / 64][kPeakStage];
    __shared__ float s_win[LDS ? kPeakTile + 2 * kPeakLdsRadius : 1];
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
    const int64_t r = a.radius;
    for (int64_t t = blockIdx.x; t * kPeakTile < len; t += gridDim.x) {
        const int64_t t0 = t * kPeakTile;
        const int64_t w0 = t0 - r > 0 ? t0 - r : 0;                              // window of the tile
        const int64_t w1 = t0 + kPeakTile + r < len ? t0 + kPeakTile + r : len;
        float v[kPeakPer];
        int hv[kPeakPer];
#pragma unroll
        for (int i = 0; i < kPeakPer; ++i) {
            const int64_t n = t0 + threadIdx.x + (int64_t)i * kBlock;
            v[i] = n < len ? snr[n] : 0.0f;
            hv[i] = n < len ? harm[n] : 0;
        }
        if constexpr (LDS) {
            __syncthreads();                                                      // previous tile done with s_win
            for (int64_t j = w0 + threadIdx.x; j < w1; j += kBlock) s_win[j - w0] = snr[j];
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < kPeakPer; ++i) {
            const int64_t n = t0 + threadIdx.x + (int64_t)i * kBlock;
            bool keep = n < len && v[i] > a.thr && hv[i] > 0;
            if (keep) {
                // beaten by an equal or larger SNR on the left, a larger one on
                // the right; no early exit, so the window reads pipeline
                const int64_t lo = n - r > 0 ? n - r : 0;
                const int64_t hi = n + r + 1 < len ? n + r + 1 : len;
                bool beaten = false;
                if constexpr (LDS) {
                    const float *wl = s_win - w0;
#pragma unroll 4
                    for (int64_t j = lo; j < n; ++j) beaten |= wl[j] >= v[i];
#pragma unroll 4
                    for (int64_t j = n + 1; j < hi; ++j) beaten |= wl[j] > v[i];
                } else {
                    for (int64_t j = lo; j < n && !beaten; ++j) beaten = snr[j] >= v[i];
                    for (int64_t j = n + 1; j < hi && !beaten; ++j) beaten = snr[j] > v[i];
                }
                keep = !beaten;
            }
            hs_candidate rec;
            rec.spectrum = (uint32_t)sp;
            rec.bin = (uint32_t)n;
            rec.snr = v[i];
            rec.harm = (uint16_t)hv[i];
            rec.drift = (uint16_t)(keep && a.drift ? a.drift[off + n] : 0);
            stage_push<kPeakStage>(st, a.cand, a.cap, a.count, keep, rec);
        }
    }
    stage_flush_block<kBlock / 64>(st, a.cand, a.cap, a.count);
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

// Each wave ends with one atomic on the shared candidate counter when it holds
// records, and those atomics serialise on one address: about 4096 workgroups
// in all, each looping over tiles (131k one-tile waves cost 1.3 ms in flushes
// on the 2^27-bin batch, against 0.2 ms here).
constexpr int64_t kPeakBlocks = 4096;

hipError_t launch_peaks(const PeakArgs &a, int groups, int64_t max_len, hipStream_t st) {
    int64_t per = (max_len + kPeakTile - 1) / kPeakTile;
    const int64_t cap = (kPeakBlocks + groups - 1) / groups;
    if (per > cap) per = cap;
    if (per < 1) per = 1;
    if (a.radius <= kPeakLdsRadius)
        hipLaunchKernelGGL(k_peaks<true>, dim3((unsigned)per, (unsigned)groups), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL(k_peaks<false>, dim3((unsigned)per, (unsigned)groups), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace hs
