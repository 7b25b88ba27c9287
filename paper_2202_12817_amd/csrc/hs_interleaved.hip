// Interleaved multi-spectrum layout (gfx950): the transposed layout of
// Sec. 3.1.1, in which the same bin of different spectra lies side by side.
// B equal-length spectra of N bins are stored as x[m B + s] (bin m of
// spectrum s).  The sums are those of Sec. 3.1 Eq. (3) and Sec. 3.3 Eq. (5) /
// Algorithm 2 per spectrum, normalised per spectrum (Eq. (2)); only the
// mapping onto the machine differs:
//
//   * a wave's 64 lanes are 64 spectra at the same fundamental n, so the
//     harmonic row k n is wave-uniform: its byte offset is a scalar (SGPR)
//     carried by one scalar addition per harmonic, and the simple sum's read
//     of harmonic k is one contiguous 64-element row segment (256 B in FP32)
//     instead of a stride-k gather;
//   * the greedy drift is per spectrum, so the greedy pair sits at rows
//     k n + d_s and k n + d_s + 1 (a per-lane row offset added to the scalar
//     one); lanes with the same drift share cache lines;
//   * the lanes read their spectra's (rs_k, nm_k) from a copy of the tables
//     stored spectrum-fastest (one coalesced 64-entry row per harmonic,
//     shared by the fundamentals walked together);
//   * the number of harmonics K(n) = min(H, (N-1) / (n + greedy)) is the same
//     for every lane and only falls as n grows: it is walked down per
//     fundamental instead of divided.
//
// Statistics (Eq. (2), a1): lane = spectrum; each thread accumulates its
// spectrum's rows of one chunk in double-double (the same exact-in-practice
// sums as for the contiguous layout, so the rounded statistics are
// identical); the chunk partials go to the shared finalise kernel.
#include "hs_internal.h"

namespace hs {
namespace {

template <bool F16>
__device__ __forceinline__ float load_off(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (F16) {
        unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
        return (float)__builtin_bit_cast(_Float16, b);
    } else {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    }
}

// Chunk c (blockIdx.x) of the rows [first_bin, N) of the spectra
// blockIdx.y * kBlock + threadIdx.x.
template <bool F16>
__global__ __launch_bounds__(kBlock) void k_stats_il(StatsArgs a) {
    constexpr uint32_t eb = F16 ? 2u : 4u;
    const int B = a.il_spectra;
    const int s = blockIdx.y * kBlock + threadIdx.x;
    if (s >= B) return;
    const int c = blockIdx.x;
    const int64_t f0 = a.first_bin;
    const int64_t W = a.n_bins > f0 ? a.n_bins - f0 : 0;
    const int64_t r_lo = f0 + W * c / a.chunks, r_hi = f0 + W * (c + 1) / a.chunks;
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(a.x, (uint32_t)(a.n_bins * B * eb));
    const uint32_t rb = (uint32_t)B * eb;
    const uint32_t voff = (uint32_t)s * eb;
    dd s1{0.0, 0.0}, s2{0.0, 0.0};
    uint32_t soff = (uint32_t)(r_lo * rb);
    int64_t r = r_lo;
    for (; r + 4 <= r_hi; r += 4, soff += 4 * rb) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = load_off<F16>(rsrc, voff, soff + (uint32_t)j * rb);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double x = (double)v[j];
            s1 = dd_add_d(s1, x);
            s2 = dd_add_d(s2, x * x);      // the square of a float is exact in double
        }
    }
    for (; r < r_hi; ++r, soff += rb) {
        const double x = (double)load_off<F16>(rsrc, voff, soff);
        s1 = dd_add_d(s1, x);
        s2 = dd_add_d(s2, x * x);
    }
    a.parts[(int64_t)s * a.chunks + c] = StatPart{s1.hi, s1.lo, s2.hi, s2.lo};
}

constexpr int kIlStage = 64;   // candidate records staged per wave
// fundamentals walked together by a wave: their loads (and the greedy
// dependency chains) overlap
template <bool GREEDY>
constexpr int il_chains() { return GREEDY ? 4 : 4; }

// One wave task: spectra group g (lanes = spectra 64 g .. 64 g + 63) x
// fundamentals [n_lo, n_lo + tile).  Workgroup L (renumbered as in
// batched_block) runs tasks 4 L .. 4 L + 3, group fastest.
template <int HMAX, bool GREEDY, bool F16>
__global__ __launch_bounds__(kBlock) void k_sum_il(IlArgs a) {
    constexpr uint32_t eb = F16 ? 2u : 4u;
    constexpr int kIlChains = il_chains<GREEDY>();
    __shared__ hs_candidate s_stage[kBlock / 64][kIlStage];
    Stage st{s_stage[threadIdx.x >> 6], 0};
    int bx, by;
    batched_block(a.n_xcd, &bx, &by);
    const int64_t task = ((int64_t)by * gridDim.x + bx) * (kBlock / 64) + (threadIdx.x >> 6);
    if (task >= a.n_tasks) return;                  // wave-uniform: the whole wave leaves
    const int lane = threadIdx.x & 63;
    const int g = (int)(task % a.n_groups);
    const int64_t N = a.n_bins;
    const int64_t n_lo = (task / a.n_groups) * a.tile;
    const int64_t n_hi = n_lo + a.tile < N ? n_lo + a.tile : N;
    const int B = a.n_spectra;
    const int s = g * 64 + lane;
    const bool live = s < B;
    const int sc = live ? s : B - 1;
    const int valid = live ? a.norm[sc].valid : 0;
    const float2 *tab = a.tab_t + sc;           // (rs_k, nm_k) at tab[(k-1) tab_stride]: one coalesced row per k
    const uint32_t rb = (uint32_t)B * eb;                       // bytes per row (bin)
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(a.x, (uint32_t)(N * B * eb));
    // lanes past the last spectrum read the last spectrum's column (never
    // written out), so every address stays inside the array
    const uint32_t vlane = (uint32_t)sc * eb;
    const int64_t n_end = a.n_end < N ? a.n_end : N;
    const int64_t gr = GREEDY ? 1 : 0;
    int K = a.H;
    {
        const int64_t n0 = n_lo > 1 ? n_lo : 1;
        const int64_t kk = (N - 1) / (n0 + gr);
        if (kk < K) K = (int)kk;
    }
    // kIlChains consecutive fundamentals walk together, so their loads (and
    // the greedy dependency chains) overlap; K is the same for every lane
    for (int64_t n0 = n_lo; n0 < n_hi; n0 += kIlChains) {
        int Kn[kIlChains];
        float S[kIlChains], best[kIlChains];
        int kb[kIlChains], db[kIlChains], d[kIlChains];
        uint32_t dv[kIlChains], step[kIlChains], srow[kIlChains];
#pragma unroll
        for (int j = 0; j < kIlChains; ++j) {
            const int64_t n = n0 + j;
            Kn[j] = 0;
            if (n < n_hi && n >= a.first_bin && n < n_end) {
                while (K > 0 && (int64_t)K * (n + gr) > N - 1) --K;     // K(n), wave-uniform
                Kn[j] = K;
            }
            S[j] = 0.0f;
            best[j] = 0.0f;
            kb[j] = db[j] = d[j] = 0;
            dv[j] = 0;                                  // d rb
            step[j] = (uint32_t)(n < n_hi ? n : 0) * rb;   // n rb < N B eb < 2^32
            srow[j] = 0;
        }
        int Kmax = 0;                                   // chains below first_bin or past the end have K = 0
#pragma unroll
        for (int j = 0; j < kIlChains; ++j) Kmax = Kn[j] > Kmax ? Kn[j] : Kmax;
#pragma unroll
        for (int k = 1; k <= HMAX; ++k) {
            if (k > Kmax) break;                        // wave-uniform
            float v[kIlChains];
#pragma unroll
            for (int j = 0; j < kIlChains; ++j) {
                srow[j] += step[j];                     // row k n, scalar
                if (k <= Kn[j]) {                       // wave-uniform
                    if constexpr (GREEDY) {
                        const float x0 = load_off<F16>(rsrc, vlane + dv[j], srow[j]);
                        const float x1 = load_off<F16>(rsrc, vlane + dv[j], srow[j] + rb);
                        const bool up = x1 > x0;
                        v[j] = up ? x1 : x0;
                        dv[j] += up ? rb : 0u;
                        d[j] += up ? 1 : 0;
                    } else {
                        v[j] = load_off<F16>(rsrc, vlane, srow[j]);
                    }
                }
            }
            const float2 t = tab[(int64_t)(k - 1) * a.tab_stride];
#pragma unroll
            for (int j = 0; j < kIlChains; ++j) {
                if (k <= Kn[j]) {
                    S[j] = S[j] + v[j];
                    const float snr = __builtin_fmaf(S[j], t.x, t.y);
                    if ((a.kmask >> (k - 1)) & 1ull) {
                        if (kb[j] == 0 || snr > best[j]) {
                            best[j] = snr;
                            kb[j] = k;
                            db[j] = d[j];
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kIlChains; ++j) {
            const int64_t n = n0 + j;
            if (n >= n_hi) continue;                    // wave-uniform
            const int kbj = valid ? kb[j] : 0;
            const float o_snr = kbj ? best[j] : 0.0f;
            const int64_t o = n * B + s;
            if (live) {
                if (a.snr) a.snr[o] = o_snr;
                if (a.harm) a.harm[o] = (uint8_t)kbj;
                if (a.drift) a.drift[o] = (uint8_t)(kbj ? db[j] : 0);
            }
            if (a.cand) {
                hs_candidate rec;
                rec.spectrum = (uint32_t)s;
                rec.bin = (uint32_t)n;
                rec.snr = o_snr;
                rec.harm = (uint16_t)kbj;
                rec.drift = (uint16_t)(kbj ? db[j] : 0);
                stage_push<kIlStage>(st, a.cand, a.cap, a.count, live && kbj > 0 && o_snr > a.thr, rec);
            }
        }
    }
    if (a.cand) stage_flush(st, a.cand, a.cap, a.count);
}

// [B][N] -> [N][B] through a 64 x 64 LDS tile: block (64, 4) threads, tile
// (blockIdx.x: bins, blockIdx.y: spectra); reads rows of one spectrum and
// writes rows of one bin, both contiguous.
template <typename T>
__global__ __launch_bounds__(256) void k_interleave(const T *__restrict__ x, int64_t N, int B, T *__restrict__ out) {
    __shared__ T tile[64][65];
    const int64_t n0 = (int64_t)blockIdx.x * 64;
    const int s0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int j = ty; j < 64; j += 4) {
        const int s = s0 + j;
        const int64_t n = n0 + tx;
        if (s < B && n < N) tile[j][tx] = x[(int64_t)s * N + n];
    }
    __syncthreads();
    for (int j = ty; j < 64; j += 4) {
        const int64_t n = n0 + j;
        const int s = s0 + tx;
        if (s < B && n < N) out[n * B + s] = tile[tx][j];
    }
}

template <int HMAX>
hipError_t sum_il_h(const IlArgs &a, bool greedy, bool f16, dim3 grid, hipStream_t st) {
    if (greedy) {
        if (f16)
            hipLaunchKernelGGL((k_sum_il<HMAX, true, true>), grid, dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_sum_il<HMAX, true, false>), grid, dim3(kBlock), 0, st, a);
    } else {
        if (f16)
            hipLaunchKernelGGL((k_sum_il<HMAX, false, true>), grid, dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_sum_il<HMAX, false, false>), grid, dim3(kBlock), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stats_il(const StatsArgs &a, bool f16, hipStream_t st) {
    dim3 grid(a.chunks, (a.il_spectra + kBlock - 1) / kBlock);
    if (f16)
        hipLaunchKernelGGL(k_stats_il<true>, grid, dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL(k_stats_il<false>, grid, dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sum_il(const IlArgs &a, int hmax, bool greedy, bool f16, hipStream_t st) {
    // tasks of 4 waves per workgroup; blocks on a 2D grid (x <= 65535 each row)
    const int64_t blocks = (a.n_tasks + kBlock / 64 - 1) / (kBlock / 64);
    const int64_t gx = blocks < 32768 ? blocks : 32768;
    const int64_t gy = (blocks + gx - 1) / gx;
    dim3 grid((unsigned)gx, (unsigned)gy);
    switch (hmax) {
        case 4: return sum_il_h<4>(a, greedy, f16, grid, st);
        case 8: return sum_il_h<8>(a, greedy, f16, grid, st);
        case 16: return sum_il_h<16>(a, greedy, f16, grid, st);
        case 32: return sum_il_h<32>(a, greedy, f16, grid, st);
        case 64: return sum_il_h<64>(a, greedy, f16, grid, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_interleave(const void *x, int64_t n_bins, int n_spectra, int elem_bytes, void *out, hipStream_t st) {
    dim3 grid((unsigned)((n_bins + 63) / 64), (unsigned)((n_spectra + 63) / 64));
    if (elem_bytes == 2)
        hipLaunchKernelGGL(k_interleave<uint16_t>, grid, dim3(256), 0, st, (const uint16_t *)x, n_bins, n_spectra,
                           (uint16_t *)out);
    else
        hipLaunchKernelGGL(k_interleave<uint32_t>, grid, dim3(256), 0, st, (const uint32_t *)x, n_bins, n_spectra,
                           (uint32_t *)out);
    return hipGetLastError();
}

}  // namespace hs
