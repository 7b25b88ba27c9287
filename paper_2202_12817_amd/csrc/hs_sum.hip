// Harmonic-sum kernels (gfx950).
//
// One lane owns one fundamental bin n and walks its harmonics k = 1..K in
// order (the per-fundamental procedure of Sec. 3.1 Eq. (3) and Sec. 3.3
// Eq. (5) / Algorithm 2):
//   simple: v = x[k n]
//   greedy: a = x[k n + d], b = x[k n + d + 1]; b > a ? (d++, v = b) : v = a
//   S += v (float, harmonic order); snr = fma(S, rs_k, nm_k)  (Eq. (2))
//   best: strictly larger SNR among the k selected by the mask.
// Consecutive lanes own consecutive fundamentals, so harmonic k of a wave
// reads a window of 64 k bins (strided by k); the greedy pair is one 8-byte
// buffer load.  The normalisation table is wave-uniform and read with
// scalar loads.  K = min(H, (N-1) / (n + greedy)) keeps every read inside
// the spectrum; the buffer descriptors additionally bound every read by the
// spectrum's size.  A wave whose 64 fundamentals share K (almost all of
// them) takes walk_uniform, without per-lane bounds; the others take walk.
#include "hs_internal.h"

namespace hs {
namespace {

// Harmonic walk of fundamental n of one spectrum (descriptor r); K harmonics.
// REPORT: also store S_k for the k in report_mask (slot-major, stride pstride).
template <int HMAX, bool GREEDY, bool F16, bool REPORT>
__device__ __forceinline__ Best walk(__amdgpu_buffer_rsrc_t r, uint32_t n, int K, const ctab_t *tab,
                                     uint64_t kmask, uint64_t report_mask, float *partial, int64_t pstride) {
    using L = Loader<F16>;
    float S = 0.0f, best = 0.0f;
    int kb = 0, db = 0;
    uint32_t d = 0;
    uint32_t m = n;   // k n
#pragma unroll
    for (int k = 1; k <= HMAX; ++k) {
        if (k > K) break;
        float v;
        if constexpr (GREEDY) {
            const float2 p = L::two(r, m + d);
            const bool up = p.y > p.x;
            v = up ? p.y : p.x;
            d += up ? 1u : 0u;
        } else {
            v = L::one(r, m);
        }
        S = S + v;
        const float2 t = tab_at(tab, k);
        const float snr = __builtin_fmaf(S, t.x, t.y);
        if constexpr (REPORT) {
            if ((report_mask >> (k - 1)) & 1ull) {
                const int slot = __builtin_popcountll(report_mask & ((1ull << (k - 1)) - 1ull));
                partial[slot * pstride] = S;
            }
        }
        if ((kmask >> (k - 1)) & 1ull) {
            if (kb == 0 || snr > best) {
                best = snr;
                kb = k;
                db = (int)d;
            }
        }
        m += n;
    }
    return Best{kb ? best : 0.0f, kb, db};
}

// C consecutive harmonics k..k+C-1 of a simple sum: all C loads first, then
// their updates in harmonic order.
template <int C, bool F16, class RowOf, class Upd>
__device__ __forceinline__ void simple_block(int k, uint32_t &md, uint32_t n, RowOf &row, Upd &update) {
    float v[C];
#pragma unroll
    for (int j = 0; j < C; ++j) v[j] = Loader<F16>::one(row(k + j), md + (uint32_t)j * n);
#pragma unroll
    for (int j = 0; j < C; ++j) update(k + j, v[j], 0u);
    md += (uint32_t)C * n;
}

// Walk of a fundamental whose wave sums the same number of harmonics KU on
// every lane, all of them eligible (the common case: K changes only where
// (len - 1) / (n + greedy) crosses an integer, and a wave holds 64
// consecutive fundamentals).  No per-lane bound or eligibility test: every
// step loads, selects and updates.  The greedy walk keeps one index per
// fundamental, md = k n + d (the left element of harmonic k's pair, in the
// row row(k) reads), advanced by n + up; the drift at the best harmonic
// comes from the index after that step, d = md' - (kb + 1) n.  Same sums,
// SNRs and comparisons as walk().
template <int HMAX, bool GREEDY, bool F16, class RowOf>
__device__ __forceinline__ Best walk_uniform(uint32_t n, int KU, const ctab_t *tab, RowOf row) {
    using L = Loader<F16>;
    float S = 0.0f, best = 0.0f;
    int kb = 0;
    uint32_t md = n, mdb = 0;
    auto update = [&](int k, float v, uint32_t nx) {
        S = S + v;
        const float2 t = tab_at(tab, k);
        const float snr = __builtin_fmaf(S, t.x, t.y);
        const bool upd = k == 1 || snr > best;              // the first eligible k, then strict >
        best = upd ? snr : best;
        kb = upd ? k : kb;
        if constexpr (GREEDY) mdb = upd ? nx : mdb;
    };
    if constexpr (GREEDY) {
#pragma unroll
        for (int k = 1; k <= HMAX; ++k) {
            if (k > KU) break;                              // wave-uniform
            const float2 p = L::two(row(k), md);
            const bool up = p.y > p.x;
            const uint32_t nx = md + n + (up ? 1u : 0u);
            update(k, up ? p.y : p.x, nx);
            md = nx;
        }
    } else {
        // the reads do not depend on the data: groups of harmonics are loaded
        // together (one basic block; eight loads in flight in the buckets of
        // 32 and 64 harmonics, where the lowest fundamentals' 32-step walks
        // set a single spectrum's time, four in the smaller buckets, where
        // eight measured slower on the plane), then the one to three left
        // over, again together
        int k = 1;
        if constexpr (HMAX >= 32) {
            while (k + 7 <= KU) {                           // wave-uniform
                simple_block<8, F16>(k, md, n, row, update);
                k += 8;
            }
            if (k + 3 <= KU) {
                simple_block<4, F16>(k, md, n, row, update);
                k += 4;
            }
        } else {
            while (k + 3 <= KU) {                           // wave-uniform
                simple_block<4, F16>(k, md, n, row, update);
                k += 4;
            }
        }
        const int r = KU - k + 1;
        if (r == 3)
            simple_block<3, F16>(k, md, n, row, update);
        else if (r == 2)
            simple_block<2, F16>(k, md, n, row, update);
        else if (r == 1)
            simple_block<1, F16>(k, md, n, row, update);
    }
    return Best{kb ? best : 0.0f, kb, (GREEDY && kb) ? (int)(mdb - (uint32_t)(kb + 1) * n) : 0};
}

// Candidate records staged per wave in LDS before one global atomic per
// flush (a device-wide atomic per wave step serialises on one address).
constexpr int kPlainStage = 64;

// 1D spectra: workgroup -> (tile block bx, spectrum s) by batched_block
// (s = 0 for one spectrum); tiles of kBlock fundamentals, tile
// t = bx + j gridDim.x.
template <int HMAX, bool GREEDY, bool F16>
__global__ __launch_bounds__(kBlock) void k_sum_1d(SumArgs a) {
    constexpr uint32_t eb = Loader<F16>::kBytes;
    __shared__ hs_candidate s_stage[kBlock / 64][kPlainStage];
    Stage st{s_stage[threadIdx.x >> 6], 0};
    int bx, s;
    batched_block(a.n_xcd, &bx, &s);
    int64_t off = 0, len = a.n_bins;
    if (a.offsets) {
        off = a.offsets[s];
        len = a.offsets[s + 1] - off;
        if (len < 0 || len >= (1ll << 30)) len = 0;   // malformed offsets: no output, no read
    }
    const NormRec *nr = a.norm + s;
    const int valid = nr->valid;
    const ctab_t *tab = const_table(nr->t);
    const char *base = (const char *)a.x + off * eb;
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(base, (uint32_t)(len * eb));
    const int64_t n_end = a.n_end < len ? a.n_end : len;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int32_t thr = k_threshold<GREEDY>(len, a.H);
    // tiles past n_end hold no fundamental: only dense outputs need them (zeros)
    const int64_t t_lim = (a.snr || a.harm || a.drift || a.partial) ? len : n_end;
    for (int64_t t = bx; t * kBlock < t_lim; t += gridDim.x) {
        const int64_t n = t * kBlock + threadIdx.x;
        const bool in = n < len;
        const int KU = (valid && a.partial == nullptr)
                           ? uniform_k(thr, t * kBlock + w * 64, t * kBlock + w * 64 + 63, a.first_bin, n_end, a.kmask)
                           : 0;
        Best b;
        int K = 0;
        if (KU == 0 && in && valid && n >= a.first_bin && n < n_end) {
            // 32-bit: len < 2^30
            const uint32_t kk = (uint32_t)(len - 1) / (uint32_t)(GREEDY ? n + 1 : n);
            K = kk < (uint32_t)a.H ? (int)kk : a.H;
        }
        if (KU > 0) {
            b = walk_uniform<HMAX, GREEDY, F16>((uint32_t)n, KU, tab, [&](int) { return rsrc; });
        } else if (a.partial == nullptr) {
            b = walk<HMAX, GREEDY, F16, false>(rsrc, (uint32_t)n, K, tab, a.kmask, 0, nullptr, 0);
        } else {
            float *prow = a.partial + off + n;
            if (in)
                for (uint64_t rm = a.report_mask, slot = 0; rm; rm &= rm - 1, ++slot) prow[slot * len] = 0.0f;
            b = walk<HMAX, GREEDY, F16, true>(rsrc, (uint32_t)n, K, tab, a.kmask, a.report_mask, prow, len);
        }
        if (in) {   // outputs are never read again: non-temporal stores
            if (a.snr) __builtin_nontemporal_store(b.snr, a.snr + off + n);
            if (a.harm) __builtin_nontemporal_store((uint8_t)b.harm, a.harm + off + n);
            if (a.drift) __builtin_nontemporal_store((uint8_t)b.drift, a.drift + off + n);
        }
        if (a.cand) {
            hs_candidate rec;
            rec.spectrum = (uint32_t)s;
            rec.bin = (uint32_t)n;
            rec.snr = b.snr;
            rec.harm = (uint16_t)b.harm;
            rec.drift = (uint16_t)b.drift;
            stage_push<kPlainStage>(st, a.cand, a.cap, a.count, in && b.harm > 0 && b.snr > a.thr, rec);
        }
    }
    if (a.cand) stage_flush_block<kBlock / 64>(st, a.cand, a.cap, a.count);
}

// Outputs of fundamental r of plane row i (dense arrays and/or staged
// candidate records; the bin of a record is i n_r + r).
__device__ __forceinline__ void plane_out(const Sum2dArgs &a, int i, int64_t r, bool in, const Best &b, Stage &st) {
    const int64_t o = (int64_t)i * a.n_r + r;
    if (in) {   // outputs are never read again: non-temporal, so they do not crowd the rows out of L2
        if (a.snr) __builtin_nontemporal_store(b.snr, a.snr + o);
        if (a.harm) __builtin_nontemporal_store((uint8_t)b.harm, a.harm + o);
        if (a.drift) __builtin_nontemporal_store((uint8_t)b.drift, a.drift + o);
    }
    if (a.cand) {
        hs_candidate rec;
        rec.spectrum = 0u;
        rec.bin = (uint32_t)o;
        rec.snr = b.snr;
        rec.harm = (uint16_t)b.harm;
        rec.drift = (uint16_t)b.drift;
        stage_push<kPlainStage>(st, a.cand, a.cap, a.count, in && b.harm > 0 && b.snr > a.thr, rec);
    }
}

// One column tile of row i: lane owns fundamental r.
template <int HMAX, bool GREEDY, bool F16>
__device__ __forceinline__ void walk_2d_tile(const Sum2dArgs &a, int i, int z, int kz, int64_t rt, int valid,
                                             const ctab_t *tab, int32_t thr, Stage &st) {
    using L = Loader<F16>;
    constexpr uint32_t eb = L::kBytes;
    const int64_t r = rt + threadIdx.x;
    const bool in = r < a.n_r;
    const int64_t n_end = a.n_end < a.n_r ? a.n_end : a.n_r;
    const uint32_t row_bytes = (uint32_t)(a.n_r * eb);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int KU = valid ? uniform_k(thr, rt + w * 64, rt + w * 64 + 63, a.first_bin, n_end, a.kmask) : 0;
    if (KU > 0) {
        // harmonic k reads row k z: its descriptor is wave-uniform (scalar)
        const Best b = walk_uniform<HMAX, GREEDY, F16>((uint32_t)r, KU, tab, [&](int k) {
            const int64_t row = (int64_t)k * z - a.z_min;
            return make_rsrc((const char *)a.plane + row * a.stride * eb, row_bytes);
        });
        plane_out(a, i, r, true, b, st);   // KU > 0: every lane of the wave is inside the row
        return;
    }
    int K = 0;
    if (in && valid && r >= a.first_bin && r < n_end) {
        const uint32_t kk = (uint32_t)(a.n_r - 1) / (uint32_t)(GREEDY ? r + 1 : r);   // n_r < 2^30
        K = kk < (uint32_t)kz ? (int)kk : kz;
    }
    float S = 0.0f, best = 0.0f;
    int kb = 0, db = 0;
    uint32_t d = 0, m = (uint32_t)r;
#pragma unroll
    for (int k = 1; k <= HMAX; ++k) {
        if (k > K) break;
        const int64_t row = (int64_t)k * z - a.z_min;    // inside [0, n_z) for k <= kz
        const __amdgpu_buffer_rsrc_t rs = make_rsrc((const char *)a.plane + row * a.stride * eb, row_bytes);
        float v;
        if constexpr (GREEDY) {
            float2 p = L::two(rs, m + d);
            bool up = p.y > p.x;
            v = up ? p.y : p.x;
            d += up ? 1u : 0u;
        } else {
            v = L::one(rs, m);
        }
        S = S + v;
        const float2 t = tab_at(tab, k);
        const float snr = __builtin_fmaf(S, t.x, t.y);
        if ((a.kmask >> (k - 1)) & 1ull) {
            if (kb == 0 || snr > best) {
                best = snr;
                kb = k;
                db = (int)d;
            }
        }
        m += (uint32_t)r;
    }
    plane_out(a, i, r, in, Best{kb ? best : 0.0f, kb, db}, st);
}

// f-fdot plane: blockIdx.y = row i - row0 (z = z_min + i); column tiles of
// kBlock fundamentals, tile t = blockIdx.x + j gridDim.x.
template <int HMAX, bool GREEDY, bool F16>
__global__ __launch_bounds__(kBlock) void k_sum_2d(Sum2dArgs a) {
    __shared__ hs_candidate s_stage[kBlock / 64][kPlainStage];
    Stage st{s_stage[threadIdx.x >> 6], 0};
    const int i = a.row0 + (int)blockIdx.y;
    const int z = a.z_min + i;
    const NormRec *nr = a.norm;
    const int valid = nr->valid;
    const ctab_t *tab = const_table(nr->t);
    int kz = a.H;
    if (z > 0) kz = a.z_max / z;
    if (z < 0) kz = a.z_min / z;
    if (kz > a.H) kz = a.H;
    const int32_t thr = k_threshold<GREEDY>(a.n_r, kz);
    const int64_t t_lim = (a.snr || a.harm || a.drift) ? a.n_r : (a.n_end < a.n_r ? a.n_end : a.n_r);
    for (int64_t t = blockIdx.x; t * kBlock < t_lim; t += gridDim.x)
        walk_2d_tile<HMAX, GREEDY, F16>(a, i, z, kz, t * kBlock, valid, tab, thr, st);
    if (a.cand) stage_flush_block<kBlock / 64>(st, a.cand, a.cap, a.count);
}

template <int HMAX>
hipError_t sum1d_h(const SumArgs &a, bool greedy, bool f16, dim3 grid, hipStream_t st) {
    if (greedy) {
        if (f16)
            hipLaunchKernelGGL((k_sum_1d<HMAX, true, true>), grid, dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_sum_1d<HMAX, true, false>), grid, dim3(kBlock), 0, st, a);
    } else {
        if (f16)
            hipLaunchKernelGGL((k_sum_1d<HMAX, false, true>), grid, dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_sum_1d<HMAX, false, false>), grid, dim3(kBlock), 0, st, a);
    }
    return hipGetLastError();
}

template <int HMAX>
hipError_t sum2d_h(const Sum2dArgs &a, bool greedy, bool f16, dim3 grid, hipStream_t st) {
    if (greedy) {
        if (f16)
            hipLaunchKernelGGL((k_sum_2d<HMAX, true, true>), grid, dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_sum_2d<HMAX, true, false>), grid, dim3(kBlock), 0, st, a);
    } else {
        if (f16)
            hipLaunchKernelGGL((k_sum_2d<HMAX, false, true>), grid, dim3(kBlock), 0, st, a);
        else
            hipLaunchKernelGGL((k_sum_2d<HMAX, false, false>), grid, dim3(kBlock), 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sum_1d(const SumArgs &a, int hmax, bool greedy, bool f16, dim3 grid, hipStream_t st) {
    switch (hmax) {
        case 4: return sum1d_h<4>(a, greedy, f16, grid, st);
        case 8: return sum1d_h<8>(a, greedy, f16, grid, st);
        case 16: return sum1d_h<16>(a, greedy, f16, grid, st);
        case 32: return sum1d_h<32>(a, greedy, f16, grid, st);
        case 64: return sum1d_h<64>(a, greedy, f16, grid, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sum_2d(const Sum2dArgs &a, int hmax, bool greedy, bool f16, int rows, hipStream_t st) {
    // about kPlainBlocks workgroups in all, each looping over column tiles
    const int64_t tiles = (a.n_r + kBlock - 1) / kBlock;
    int64_t per_row = (kPlainBlocks + rows - 1) / rows;
    if (per_row > tiles) per_row = tiles;
    dim3 grid((unsigned)per_row, (unsigned)rows);
    switch (hmax) {
        case 4: return sum2d_h<4>(a, greedy, f16, grid, st);
        case 8: return sum2d_h<8>(a, greedy, f16, grid, st);
        case 16: return sum2d_h<16>(a, greedy, f16, grid, st);
        case 32: return sum2d_h<32>(a, greedy, f16, grid, st);
        case 64: return sum2d_h<64>(a, greedy, f16, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hs
