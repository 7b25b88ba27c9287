// PRESTO-style harmonic sums (gfx950): the comparators of Sec. 3.2 (Eq. (4),
// Algorithm 1).  The output index n is the LAST bin of a harmonic series:
// stage K (harmonic order K) sums the bins nearest to h n / K (halves rounded
// up) for its harmonics h, in increasing h, and forms one SNR (Eq. (2)) from
// the stage's m-element sum:
//   HS_PRESTO:      K = 2, 4, 8, ...; h = 1 and the even h <= K; m = 1 + K/2
//   HS_PRESTO_ALL:  K = 2, 4, 8, ...; h = 1..K;                    m = K
//   HS_PRESTO_PLUS: K = 1..H;         h = 1..K;                    m = K
// A stage is formed only while its fundamental, the bin nearest to n / K, is
// >= first_bin (it only falls as K grows, so the first unformed stage ends
// the walk); the best stage is the largest SNR among the stages the mask
// selects, ties to the smaller K.
//
// One lane owns one last bin n; consecutive lanes own consecutive bins, so a
// stage's harmonic h reads about 64 h / K consecutive bins per wave.  Stages
// share bins: the bin nearest to h n / K is bin h T / K of any stage T that
// is a multiple of K by a power of two.  So PRESTO and PRESTO_all (orders 2,
// 4, ...) read the bins of the compiled power-of-two bucket's stage once, and
// PRESTO+ groups its orders into chains o, 2 o, 4 o, ... (o odd) that read
// the bins of their top order once; every stage then sums from registers in
// increasing h (the same float sums as stage-by-stage).  With n = Q T + R
// (0 <= R < T) bin j of stage T is  j Q + floor((2 j R + T) / (2 T)):  j Q
// and 2 j R + T are carried from bin to bin by additions, and the small
// quotient (numerator <= 2 T^2 - T < 2^11) is floor(x ceil(2^20 / 2T) / 2^20),
// exact for every numerator below 2^11 and every T <= 32 (checked
// exhaustively), the high word of a 24-bit multiply (a shift when T is a
// power of two).
#include "hs_internal.h"

namespace hs {
namespace {

template <int VARIANT>
constexpr bool harmonic_summed(int h) {
    return VARIANT != HS_PRESTO || h == 1 || h % 2 == 0;
}

// floor(x / (2 K)) for x < 2^11, given x12 = x 2^12 (< 2^23): the high word
// of the 24 x 24-bit product x12 ceil(2^20 / (2 K)), one full-rate multiply.
template <int K>
__device__ __forceinline__ uint32_t div_2k(uint32_t x12) {
    constexpr uint32_t M = ((1u << 20) + 2 * K - 1) / (2 * K);
    static_assert(K >= 1 && K <= 32, "stage order out of range");
    uint32_t q;
    asm("v_mul_hi_u32_u24 %0, %1, %2" : "=v"(q) : "s"(M), "v"(x12));
    return q;
}

template <bool F16>
__device__ __forceinline__ float load_at(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    if constexpr (F16) {
        unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, (int)byte_off, 0, 0);
        return (float)__builtin_bit_cast(_Float16, b);
    } else {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
    }
}

struct StageState {
    float best;   // best SNR so far (valid when kb > 0)
    int kb;       // its stage order, 0 = none
};

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Largest o 2^e <= HMAX (the top stage of the chain of odd part o).
constexpr int chain_top(int o, int hmax) { return o * 2 > hmax ? o : chain_top(o * 2, hmax); }

// PRESTO+: the stages o, 2 o, 4 o, ... (one chain per odd o) read bins of
// their top stage T (bin h of stage K is bin h T / K of stage T), so each
// chain computes and loads T bins once and sums its stages from registers in
// h order.  Chains run in any order, so the best stage is chosen by the
// larger SNR, ties to the smaller K (the in-order rule).
template <bool F16, int O, int HMAX>
__device__ __forceinline__ void plus_chain(__amdgpu_buffer_rsrc_t r, uint32_t n, int H, uint32_t first_bin,
                                           const float2 *__restrict__ tab, uint64_t kmask, StageState &s) {
    constexpr int T = chain_top(O, HMAX);
    constexpr uint32_t eb = F16 ? 2u : 4u;
    constexpr uint32_t sh = F16 ? 1u : 2u;
    static_assert(2 * T * T - T < (1 << 11), "2 h R + T must stay below 2^11");
    if (O > H) return;
    const uint32_t fb = first_bin * eb;
    const uint32_t Q = n / (uint32_t)T;
    const uint32_t R2 = (2u * (n - Q * (uint32_t)T)) << 12;
    const uint32_t Qb = Q * eb;
    uint32_t off[T + 1];
    float v[T + 1];
    uint32_t hqb = 0, hr = (uint32_t)T << 12;
    // odd T: 2 j R + T is odd, never a multiple of 2 T, so no bin is an exact
    // half and bin T - j is n - bin j (one subtraction instead of four steps)
    constexpr int direct = (T % 2 == 1) ? (T - 1) / 2 : T;
#pragma unroll
    for (int j = 1; j <= direct; ++j) {
        hqb += Qb;
        hr += R2;
        asm("" : "+v"(hqb), "+v"(hr));
        off[j] = hqb + (div_2k<T>(hr) << sh);
    }
    if constexpr (T % 2 == 1) {
        const uint32_t nb = n * eb;
#pragma unroll
        for (int j = 1; j <= direct; ++j) off[T - j] = nb - off[j];
        off[T] = nb;
    }
#pragma unroll
    for (int j = 1; j <= T; ++j) v[j] = load_at<F16>(r, off[j]);
#pragma unroll
    for (int K = O; K <= T; K *= 2) {
        if (K > H) break;
        const int st = T / K;
        if (off[st] < fb) break;                 // fundamentals only fall as K grows
        float S = v[st];
#pragma unroll
        for (int h = 2; h <= K; ++h) S = S + v[h * st];
        const float2 t = tab[K - 1];
        const float snr = __builtin_fmaf(S, t.x, t.y);
        if ((kmask >> (K - 1)) & 1ull) {
            if (s.kb == 0 || snr > s.best || (snr == s.best && K < s.kb)) {
                s.best = snr;
                s.kb = K;
            }
        }
    }
}

template <bool F16, int O, int HMAX>
__device__ __forceinline__ void plus_chains(__amdgpu_buffer_rsrc_t r, uint32_t n, int H, uint32_t first_bin,
                                            const float2 *__restrict__ tab, uint64_t kmask, StageState &s) {
    plus_chain<F16, O, HMAX>(r, n, H, first_bin, tab, kmask, s);
    if constexpr (O + 2 <= HMAX) plus_chains<F16, O + 2, HMAX>(r, n, H, first_bin, tab, kmask, s);
}

// PRESTO and PRESTO_all: every stage order K is a power of two, so the bin
// nearest to h n / K is the bin nearest to (h HMAX / K) n / HMAX: all stages
// read bins of the HMAX stage (HMAX, the compiled bucket, is a power of two
// >= H).  Its HMAX bins are computed and loaded once (division by 2 HMAX is a
// shift) and every stage sums its elements from registers, in increasing h.
template <int VARIANT, bool F16, int HMAX>
__device__ __forceinline__ void pow2_stages(__amdgpu_buffer_rsrc_t r, uint32_t n, int H, uint32_t first_bin,
                                            const float2 *__restrict__ tab, uint64_t kmask, StageState &s) {
    static_assert((HMAX & (HMAX - 1)) == 0, "bucket must be a power of two");
    constexpr uint32_t eb = F16 ? 2u : 4u;
    constexpr uint32_t sh = F16 ? 1u : 2u;
    constexpr int lg = ilog2(2 * HMAX);
    const uint32_t Q = n >> ilog2(HMAX);
    const uint32_t R2 = 2u * (n & (uint32_t)(HMAX - 1));
    const uint32_t Qb = Q * eb;
    uint32_t off[HMAX + 1];                      // off[j]: byte offset of bin j of the HMAX stage
    float v[HMAX + 1];
    uint32_t hqb = 0, hr = (uint32_t)HMAX;       // j Q (bytes), 2 j R + HMAX
#pragma unroll
    for (int j = 1; j <= HMAX; ++j) {
        hqb += Qb;
        hr += R2;
        asm("" : "+v"(hqb), "+v"(hr));
        off[j] = hqb + ((hr >> lg) << sh);
        v[j] = load_at<F16>(r, off[j]);
    }
    const uint32_t fb = first_bin * eb;
#pragma unroll
    for (int K = 2; K <= HMAX; K *= 2) {
        if (K > H) break;
        const int st = HMAX / K;                 // bin h of stage K is bin h st of the HMAX stage
        if (off[st] < fb) break;                 // the stage's fundamental lies below first_bin
        float S = v[st];
#pragma unroll
        for (int h = 2; h <= K; ++h) {
            if (!harmonic_summed<VARIANT>(h)) continue;
            S = S + v[h * st];
        }
        const int m = VARIANT == HS_PRESTO ? 1 + K / 2 : K;
        const float2 t = tab[m - 1];
        const float snr = __builtin_fmaf(S, t.x, t.y);
        if ((kmask >> (K - 1)) & 1ull) {
            if (s.kb == 0 || snr > s.best) {
                s.best = snr;
                s.kb = K;
            }
        }
    }
}

constexpr int kPrestoStage = 64;   // candidate records staged per wave

// 1D spectra: workgroup -> (tile block bx, spectrum sp) by batched_block
// (sp = 0 for one spectrum); tiles of kBlock last bins, tile
// t = bx + j gridDim.x.
template <int HMAX, int VARIANT, bool F16>
__global__ __launch_bounds__(kBlock) void k_presto(SumArgs a) {
    constexpr uint32_t eb = F16 ? 2u : 4u;
    __shared__ hs_candidate s_stage[kBlock / 64][kPrestoStage];
    Stage st{s_stage[threadIdx.x >> 6], 0};
    int bx, sp;
    batched_block(a.n_xcd, &bx, &sp);
    int64_t off = 0, len = a.n_bins;
    if (a.offsets) {
        off = a.offsets[sp];
        len = a.offsets[sp + 1] - off;
        if (len < 0 || len >= (1ll << 30)) len = 0;   // malformed offsets: no output, no read
    }
    const NormRec *nr = a.norm + sp;
    const int valid = nr->valid;
    const float2 *tab = nr->t;
    const __amdgpu_buffer_rsrc_t rsrc = make_rsrc((const char *)a.x + off * eb, (uint32_t)(len * eb));
    const int64_t n_end = a.n_end < len ? a.n_end : len;
    for (int64_t t = bx; t * kBlock < len; t += gridDim.x) {
        const int64_t n = t * kBlock + threadIdx.x;
        const bool in = n < len;
        StageState s{0.0f, 0};
        if (in && valid && n >= a.first_bin && n < n_end) {
            if constexpr (VARIANT == HS_PRESTO_PLUS)
                plus_chains<F16, 1, HMAX>(rsrc, (uint32_t)n, a.H, (uint32_t)a.first_bin, tab, a.kmask, s);
            else
                pow2_stages<VARIANT, F16, HMAX>(rsrc, (uint32_t)n, a.H, (uint32_t)a.first_bin, tab, a.kmask, s);
        }
        const float snr = s.kb ? s.best : 0.0f;
        if (in) {
            if (a.snr) a.snr[off + n] = snr;
            if (a.harm) a.harm[off + n] = (uint8_t)s.kb;
            if (a.drift) a.drift[off + n] = 0;
        }
        if (a.cand) {
            hs_candidate rec;
            rec.spectrum = (uint32_t)sp;
            rec.bin = (uint32_t)n;
            rec.snr = snr;
            rec.harm = (uint16_t)s.kb;
            rec.drift = 0;
            stage_push<kPrestoStage>(st, a.cand, a.cap, a.count, in && s.kb > 0 && snr > a.thr, rec);
        }
    }
    if (a.cand) stage_flush_block<kBlock / 64>(st, a.cand, a.cap, a.count);
}

template <int HMAX, int VARIANT>
hipError_t presto_v(const SumArgs &a, bool f16, dim3 grid, hipStream_t st) {
    if (f16)
        hipLaunchKernelGGL((k_presto<HMAX, VARIANT, true>), grid, dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_presto<HMAX, VARIANT, false>), grid, dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

template <int HMAX>
hipError_t presto_h(const SumArgs &a, int variant, bool f16, dim3 grid, hipStream_t st) {
    switch (variant) {
        case HS_PRESTO: return presto_v<HMAX, HS_PRESTO>(a, f16, grid, st);
        case HS_PRESTO_ALL: return presto_v<HMAX, HS_PRESTO_ALL>(a, f16, grid, st);
        case HS_PRESTO_PLUS: return presto_v<HMAX, HS_PRESTO_PLUS>(a, f16, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_presto(const SumArgs &a, int hmax, int variant, bool f16, dim3 grid, hipStream_t st) {
    switch (hmax) {
        case 4: return presto_h<4>(a, variant, f16, grid, st);
        case 8: return presto_h<8>(a, variant, f16, grid, st);
        case 16: return presto_h<16>(a, variant, f16, grid, st);
        case 32: return presto_h<32>(a, variant, f16, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hs
