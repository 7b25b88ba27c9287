// Device-side helpers of the harmonic-sum library (gfx950): double-double
// arithmetic for the normalisation statistics, buffer-resource loads for the
// harmonic gathers, and the per-spectrum normalisation record.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hs.h"

namespace hs {

// Per-group (spectrum or plane) normalisation, written by the finalise kernel
// and read (wave-uniformly) by the harmonic-sum kernels.
struct NormRec {
    double mu1;        // population mean of the stored powers, rounded once
    double sigma1;     // sqrt of the population variance, rounded once
    int32_t valid;     // 0: degenerate normalisation, all outputs zero
    int32_t pad[3];
    float2 t[HS_MAX_HARMONICS];   // (rs_k, nm_k) for k = 1..HS_MAX_HARMONICS
};

// Partial statistics of one chunk: exact-in-practice double-double sums.
struct StatPart {
    double s1hi, s1lo, s2hi, s2lo;
};

// ---------------------------------------------------------------------------
// Double-double arithmetic (Knuth's TwoSum, Dekker's FastTwoSum, FMA-based
// TwoProd).  Compiled with -ffp-contract=off so every operation is the single
// IEEE rounding written here.
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    e = b - (s - a);
}

__device__ __forceinline__ dd dd_add_d(dd a, double b) {
    double s, e;
    two_sum(a.hi, b, s, e);
    e = e + a.lo;
    fast_two_sum(s, e, s, e);
    return {s, e};
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
    double s, e, t, f;
    two_sum(a.hi, b.hi, s, e);
    two_sum(a.lo, b.lo, t, f);
    e = e + t;
    fast_two_sum(s, e, s, e);
    e = e + f;
    fast_two_sum(s, e, s, e);
    return {s, e};
}

__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ dd dd_mul(dd a, dd b) {
    double p = a.hi * b.hi;
    double e = __builtin_fma(a.hi, b.hi, -p);
    double c = a.hi * b.lo;
    double c2 = a.lo * b.hi;
    e = e + (c + c2);
    double s;
    fast_two_sum(p, e, s, e);
    return {s, e};
}

// a / b for an exact double b (the element count).
__device__ __forceinline__ dd dd_div_d(dd a, double b) {
    double q1 = a.hi / b;
    double p = q1 * b;
    double pe = __builtin_fma(q1, b, -p);      // q1 * b = p + pe exactly
    dd r = dd_add(a, dd{-p, -pe});
    double q2 = r.hi / b;
    double s, e;
    fast_two_sum(q1, q2, s, e);
    return {s, e};
}

// Correctly rounded double square root: the hardware-library result is
// checked against both rounding midpoints with an exact residual and moved by
// one ulp when it is on the wrong side.
__device__ __forceinline__ double sqrt_rn(double v) {
    if (!(v > 0.0) || !__builtin_isfinite(v)) return __builtin_sqrt(v);
    double t = __builtin_sqrt(v);
    for (int it = 0; it < 2; ++it) {
        // neighbours of a positive finite double: adjacent bit patterns
        double up = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, t) + 1u);
        double dn = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, t) - 1u);
        // midpoint m = (t + up) / 2 = t + h with h = (up - t) / 2 exact (power of two)
        double h = (up - t) * 0.5;
        // v - m^2 = (v - t^2) - 2 t h - h^2, each term exact in double-double
        double p = t * t, pe = __builtin_fma(t, t, -p);
        dd r = dd_add(dd{v, 0.0}, dd{-p, -pe});
        r = dd_add_d(r, -(2.0 * t * h));
        r = dd_add_d(r, -(h * h));
        if (r.hi > 0.0 || (r.hi == 0.0 && r.lo > 0.0)) { t = up; continue; }
        double hd = (t - dn) * 0.5;
        dd q = dd_add(dd{v, 0.0}, dd{-p, -pe});
        q = dd_add_d(q, 2.0 * t * hd);
        q = dd_add_d(q, -(hd * hd));
        if (q.hi < 0.0 || (q.hi == 0.0 && q.lo < 0.0)) { t = dn; continue; }
        break;
    }
    return t;
}

// ---------------------------------------------------------------------------
// Buffer-resource loads: 32-bit byte offsets from a wave-uniform base; reads
// outside num_records return zero instead of faulting.
// ---------------------------------------------------------------------------
constexpr int32_t kRsrcFlags = 0x00020000;   // gfx9 dword3: 32-bit data format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcFlags);
}

__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, uint32_t elem) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(elem * 4u), 0, 0));
}

typedef float f32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 ld_f32x2(__amdgpu_buffer_rsrc_t r, uint32_t elem) {
    // bit-cast the whole 2-vector (a bit_cast of one element of the builtin's
    // vector result would alias element 0)
    const f32x2_t f = __builtin_bit_cast(f32x2_t, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(elem * 4u), 0, 0));
    return make_float2(f.x, f.y);
}

__device__ __forceinline__ float ld_f16(__amdgpu_buffer_rsrc_t r, uint32_t elem) {
    unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, (int)(elem * 2u), 0, 0);
    return (float)__builtin_bit_cast(_Float16, b);
}

// The greedy pair (elem, elem + 1) of 16-bit values with one 4-byte load
// (2-byte aligned when elem is odd; the memory system serves unaligned
// buffer loads): one cache-line lookup per lane instead of two.
__device__ __forceinline__ float2 ld_f16x2(__amdgpu_buffer_rsrc_t r, uint32_t elem) {
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(elem * 2u), 0, 0);
    return make_float2((float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xFFFFu)),
                       (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16)));
}

template <bool F16>
struct Loader;

template <>
struct Loader<false> {
    static constexpr uint32_t kBytes = 4;
    __device__ static float one(__amdgpu_buffer_rsrc_t r, uint32_t e) { return ld_f32(r, e); }
    __device__ static float2 two(__amdgpu_buffer_rsrc_t r, uint32_t e) { return ld_f32x2(r, e); }
};

template <>
struct Loader<true> {
    static constexpr uint32_t kBytes = 2;
    __device__ static float one(__amdgpu_buffer_rsrc_t r, uint32_t e) { return ld_f16(r, e); }
    __device__ static float2 two(__amdgpu_buffer_rsrc_t r, uint32_t e) { return ld_f16x2(r, e); }
};

// Normalisation tables are written by an earlier launch and only read by
// the sum kernels: reading them through the constant address space lets the
// compiler use scalar loads for wave-uniform indices, even in kernels that
// store to global memory (through a generic pointer it must assume the
// stores may alias the table and falls back to vector loads).
typedef __attribute__((address_space(4))) const float ctab_t;
__device__ __forceinline__ const ctab_t *const_table(const float2 *p) { return (const ctab_t *)p; }
// (rs_k, nm_k) of harmonic k of such a table
__device__ __forceinline__ float2 tab_at(const ctab_t *t, int k) { return make_float2(t[2 * k - 2], t[2 * k - 1]); }

// Harmonic counts from thresholds held one per lane.  K(n) = min(cap,
// (len - 1) / (n + greedy)) is the number of k <= cap with n <= T(k), where
// T(k) = (len - 1) / k - greedy decreases in k; lane j of every wave keeps
// T(j + 1) (-1 for j >= cap), computed once per spectrum (cap <= 64 = lanes
// of a wave), so the count of a wave-uniform n is the population of one
// ballot.  Every lane of the wave must be active when these are called.
template <bool GREEDY>
__device__ __forceinline__ int32_t k_threshold(int64_t len, int cap) {
    const int j = (int)(threadIdx.x & 63);
    if (j >= cap || len < 2) return -1;
    return (int32_t)((uint32_t)(len - 1) / (uint32_t)(j + 1)) - (GREEDY ? 1 : 0);   // len < 2^30
}

// Harmonics summed by every fundamental in [wf, wl] (wave-uniform, wl < 2^30)
// when they agree and all of them are eligible, else 0 (the caller then
// takes its walk with a bound per lane).  K is non-increasing in n, so the
// two ends decide.
__device__ __forceinline__ int uniform_k(int32_t thr, int64_t wf, int64_t wl, int64_t first_bin, int64_t n_end,
                                         uint64_t kmask) {
    // 32-bit compares (scalar): positions are below 2^30
    if ((uint32_t)wf < (uint32_t)first_bin || (uint32_t)wl >= (uint32_t)n_end) return 0;
    const int kf = __builtin_popcountll(__ballot(thr >= (int32_t)wf));
    const int kl = __builtin_popcountll(__ballot(thr >= (int32_t)wl));
    if (kf != kl || kf == 0) return 0;
    const uint64_t need = kf >= 64 ? ~0ull : (1ull << kf) - 1ull;
    return (kmask & need) == need ? kf : 0;
}

// Result of one fundamental.
struct Best {
    float snr;
    int harm;
    int drift;
};

// Per-wave candidate staging in LDS: records are appended to the wave's own
// slice (ballot + rank) and copied out with one global atomic per flush, so
// the shared counter sees one atomic per slice-full instead of one per wave
// step.  LDS writes and reads of a slice are by the same wave, ordered by the
// wave barrier in the flush.
struct Stage {
    hs_candidate *buf;    // this wave's LDS slice
    int count;            // records held (wave-uniform)
};

__device__ __forceinline__ void stage_flush(Stage &st, hs_candidate *cand, int64_t cap, unsigned long long *count) {
    if (st.count == 0) return;
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    unsigned long long cb = 0;
    if (lane == 0) cb = atomicAdd(count, (unsigned long long)st.count);
    cb = __shfl(cb, 0);
    for (int i = lane; i < st.count; i += 64)
        if ((int64_t)(cb + i) < cap) cand[cb + i] = st.buf[i];
    __builtin_amdgcn_wave_barrier();
    st.count = 0;
}

// The end of a kernel: the records still staged by the workgroup's waves are
// written with one atomic per workgroup instead of one per wave (the atomics
// of all waves serialise on the counter's address).  Every thread of the
// workgroup must call it (it synchronises the workgroup).
template <int WAVES>
__device__ __forceinline__ void stage_flush_block(Stage &st, hs_candidate *cand, int64_t cap,
                                                  unsigned long long *count) {
    __shared__ int s_cnt[WAVES];
    __shared__ unsigned long long s_base;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) s_cnt[w] = st.count;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int i = 0; i < WAVES; ++i) tot += s_cnt[i];
        s_base = tot ? atomicAdd(count, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    unsigned long long base = s_base;
    for (int i = 0; i < w; ++i) base += (unsigned long long)s_cnt[i];
    for (int i = lane; i < st.count; i += 64)
        if ((int64_t)(base + i) < cap) cand[base + i] = st.buf[i];
    st.count = 0;
}

template <int SLICE>
__device__ __forceinline__ void stage_push(Stage &st, hs_candidate *cand, int64_t cap, unsigned long long *count,
                                           bool pred, const hs_candidate &r) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const int cnt = __builtin_popcountll(mask);
    if (st.count + cnt > SLICE) stage_flush(st, cand, cap, count);
    const int lane = threadIdx.x & 63;
    if (pred) st.buf[st.count + __builtin_popcountll(mask & ((1ull << lane) - 1ull))] = r;
    st.count += cnt;
}

}  // namespace hs
