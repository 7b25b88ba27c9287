// Persistent, XCD-aware harmonic-sum kernel for batches of spectra (gfx950).
//
// Why: a fundamental's k-th harmonic reads bins near k n, so over all
// fundamentals and harmonics every cache line of a spectrum is touched about
// once per harmonic (N H s bytes for N bins of s bytes).  Whether those
// touches hit the XCD's 4 MB L2 or go to the Infinity Fabric depends only on
// scheduling: if the resident workgroups of one XCD walk one contiguous block
// of fundamentals harmonic by harmonic at the same pace, the harmonic windows
// [k a, k (a + D)] of consecutive harmonics overlap and stay in that XCD's L2.
//
// How: the grid holds as many workgroups as can be resident.  Workgroup b
// belongs to virtual XCD b % n_xcd (the hardware dispatches workgroups to XCDs
// round robin; correctness does not depend on it).  Virtual XCD q owns the
// spectra q, q + n_xcd, q + 2 n_xcd, ... and hands out their chunks of
// kBlock * F consecutive fundamentals in increasing order through one atomic
// ticket counter, so its resident workgroups always work on adjacent chunks of
// one spectrum and progress through the harmonics together.  Every ticket
// beyond the queue's last chunk ends the workgroup: all waves reach the exit.
//
// Per lane: F fundamentals (n, n + 256, ...) walked harmonic by harmonic with
// independent loads in flight.  The harmonic loop bound is wave-uniform (the
// largest K of the wave); a lane whose own K is smaller issues its loads at an
// out-of-range buffer offset, which returns zero without touching memory, and
// commits nothing.
#include "hs_internal.h"

namespace hs {
namespace {

constexpr uint32_t kOob = 0xFFFFFFF0u;   // buffer offset beyond any num_records

// Chunking of one spectrum.  Fundamentals are split into size classes j =
// 0..kClasses-1: class j covers [b_j, b_{j+1}) where b_j = (len-1)/((H>>j)+1)
// (b_0 = 0, last class up to len), so fundamentals of class j sum at most
// about H>>j harmonics; its chunks hold base << j fundamentals, keeping the
// work per chunk roughly constant.  Chunks are numbered in increasing n.
constexpr int kClasses = 6;

struct SpecInfo {
    int64_t off, len;
    uint32_t chunks;                   // total chunks of the spectrum
    uint32_t bound[kClasses + 1];      // class boundaries (fundamental index)
    uint32_t first[kClasses + 1];      // first chunk of each class
};

__device__ __forceinline__ void spec_info(SpecInfo &r, const int64_t *offsets, int s, uint32_t base, int H) {
    r.off = offsets[s];
    r.len = offsets[s + 1] - r.off;
    if (r.len < 0 || r.len >= (1ll << 30)) r.len = 0;   // malformed offsets: no output, no read
    const uint32_t len = (uint32_t)r.len;
    r.bound[0] = 0;
    r.first[0] = 0;
#pragma unroll
    for (int j = 1; j <= kClasses; ++j) {
        uint32_t b = j == kClasses ? len : (len > 0 ? (len - 1) / (uint32_t)((H >> j) + 1) : 0);
        if (b < r.bound[j - 1]) b = r.bound[j - 1];
        if (b > len) b = len;
        r.bound[j] = b;
        const uint32_t sz = base << (j - 1);
        r.first[j] = r.first[j - 1] + (r.bound[j] - r.bound[j - 1] + sz - 1) / sz;
    }
    r.chunks = r.first[kClasses];
}

// Harmonics summed by fundamental n (0 when n is no fundamental).
template <bool GREEDY>
__device__ __forceinline__ int keff(int64_t n, int64_t len, int64_t first_bin, int64_t n_end, int H) {
    if (n < first_bin || n >= n_end) return 0;
    const uint32_t kk = (uint32_t)(len - 1) / (uint32_t)(GREEDY ? n + 1 : n);
    return kk < (uint32_t)H ? (int)kk : H;
}

// Candidate staging: each wave collects its records in its own LDS slice and
// reserves space in the global list with one atomic per kStage records (a
// device-wide atomic per record would serialise the whole kernel on one
// address).  Wave-private, so no barrier is needed; the wave's LDS accesses are
// ordered by the wave barrier below.
constexpr int kStage = 256;

struct Stage {
    hs_candidate *buf;    // this wave's LDS slice [kStage]
    int count;            // records held (wave-uniform)
};

__device__ __forceinline__ void stage_flush(Stage &st, const SumArgs &a) {
    if (st.count == 0) return;
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    unsigned long long cb = 0;
    if (lane == 0) cb = atomicAdd(a.count, (unsigned long long)st.count);
    cb = __shfl(cb, 0);
    for (int i = lane; i < st.count; i += 64)
        if ((int64_t)(cb + i) < a.cap) a.cand[cb + i] = st.buf[i];
    __builtin_amdgcn_wave_barrier();
    st.count = 0;
}

__device__ __forceinline__ void stage_push(Stage &st, const SumArgs &a, bool pred, const hs_candidate &r) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const int cnt = __builtin_popcountll(mask);
    if (st.count + cnt > kStage) stage_flush(st, a);
    const int lane = threadIdx.x & 63;
    if (pred) st.buf[st.count + __builtin_popcountll(mask & ((1ull << lane) - 1ull))] = r;
    st.count += cnt;
}

// One pass: kBlock * F consecutive fundamentals starting at p0 (lane owns
// p0 + f kBlock + threadIdx.x), restricted to [p0, p_end).
template <int HMAX, bool GREEDY, bool F16, int F>
__device__ __forceinline__ void walk_pass(const SumArgs &a, int s, const SpecInfo &si, int64_t p0, int64_t p_end,
                                          __amdgpu_buffer_rsrc_t rsrc, const float2 *__restrict__ tab, int valid,
                                          Stage &st) {
    using L = Loader<F16>;
    constexpr uint32_t eb = L::kBytes;
    const int wave = threadIdx.x >> 6;
    const int64_t len = si.len;
    int64_t n_end = a.n_end < len ? a.n_end : len;
    if (p_end < n_end) n_end = p_end;
    int K[F];
    uint32_t n[F], m[F], d[F];
    float S[F], best[F];
    int kb[F], db[F];
    int KW = 0;                                             // wave-uniform loop bound
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int64_t n0 = p0 + f * kBlock;                 // first fundamental of this f-slice
        n[f] = (uint32_t)(n0 + threadIdx.x);
        K[f] = valid ? keff<GREEDY>(n0 + threadIdx.x, len, a.first_bin, n_end, a.H) : 0;
        // K is non-increasing in n: the wave's largest K is at its first fundamental >= first_bin
        int64_t nw = n0 + wave * 64;
        if (nw < a.first_bin) nw = a.first_bin;
        const int kw = valid ? keff<GREEDY>(nw, len, a.first_bin, n_end, a.H) : 0;
        KW = kw > KW ? kw : KW;
        m[f] = n[f];
        d[f] = 0;
        S[f] = 0.0f;
        best[f] = 0.0f;
        kb[f] = 0;
        db[f] = 0;
    }
#pragma unroll
    for (int k = 1; k <= HMAX; ++k) {
        if (k > KW) continue;                               // wave-uniform: skips the rest
        const float2 tk = tab[k - 1];
        const bool el = (a.kmask >> (k - 1)) & 1ull;
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const bool act = k <= K[f];
            float v;
            if constexpr (GREEDY) {
                const uint32_t o = act ? (m[f] + d[f]) * eb : kOob;
                float2 p;
                if constexpr (F16) {
                    p = make_float2(
                        (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rsrc, (int)o, 0, 0)),
                        (float)__builtin_bit_cast(_Float16,
                                                  __builtin_amdgcn_raw_buffer_load_b16(rsrc, (int)(o + 2u), 0, 0)));
                } else {
                    const f32x2_t w =
                        __builtin_bit_cast(f32x2_t, __builtin_amdgcn_raw_buffer_load_b64(rsrc, (int)o, 0, 0));
                    p = make_float2(w.x, w.y);
                }
                const bool up = p.y > p.x;                  // inactive lanes read (0, 0): no move
                v = up ? p.y : p.x;
                d[f] += up ? 1u : 0u;
            } else {
                const uint32_t o = act ? m[f] * eb : kOob;
                if constexpr (F16)
                    v = (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rsrc, (int)o, 0, 0));
                else
                    v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)o, 0, 0));
            }
            S[f] = S[f] + v;                                // + 0 on inactive lanes
            const float snr = __builtin_fmaf(S[f], tk.x, tk.y);
            const bool upd = act && el && (kb[f] == 0 || snr > best[f]);
            best[f] = upd ? snr : best[f];
            kb[f] = upd ? k : kb[f];
            db[f] = upd ? (int)d[f] : db[f];
            m[f] += n[f];
        }
    }
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const bool in = (int64_t)n[f] < p_end;
        const float bs = kb[f] ? best[f] : 0.0f;
        if (in) {
            const int64_t o = si.off + n[f];
            if (a.snr) a.snr[o] = bs;
            if (a.harm) a.harm[o] = (uint8_t)kb[f];
            if (a.drift) a.drift[o] = (uint8_t)db[f];
        }
        if (a.cand) {
            hs_candidate r;
            r.spectrum = (uint32_t)s;
            r.bin = n[f];
            r.snr = bs;
            r.harm = (uint16_t)kb[f];
            r.drift = (uint16_t)db[f];
            stage_push(st, a, in && kb[f] > 0 && bs > a.thr, r);
        }
    }
}

template <int HMAX, bool GREEDY, bool F16, int F>
__global__ __launch_bounds__(kBlock) void k_sum_xcd(XcdArgs xa) {
    constexpr uint32_t eb = Loader<F16>::kBytes;
    constexpr int CH = kBlock * F;                 // fundamentals per pass (class-0 chunk)
    const SumArgs &a = xa.s;
    const int q = blockIdx.x % xa.n_xcd;
    __shared__ uint32_t s_ticket;
    __shared__ hs_candidate s_stage[kBlock / 64][kStage];
    Stage st{s_stage[threadIdx.x >> 6], 0};

    int s = q;
    uint32_t base = 0;                              // first ticket of spectrum s
    SpecInfo si;
    si.chunks = 0;
    if (s < xa.n_spectra) spec_info(si, a.offsets, s, CH, a.H);

    if (threadIdx.x == 0) s_ticket = atomicAdd(xa.tickets + q, 1u);
    __syncthreads();
    uint32_t t = s_ticket;
    for (;;) {
        __syncthreads();                            // everyone has read s_ticket
        uint32_t next = 0;
        if (threadIdx.x == 0) next = atomicAdd(xa.tickets + q, 1u);   // prefetch: used after this chunk
        while (s < xa.n_spectra && t >= base + si.chunks) {   // advance to the spectrum holding ticket t
            base += si.chunks;
            s += xa.n_xcd;
            if (s < xa.n_spectra) spec_info(si, a.offsets, s, CH, a.H);
        }
        if (s >= xa.n_spectra) break;                          // queue exhausted (uniform)
        const uint32_t c = t - base;
        int j = 0;
        while (j + 1 < kClasses && c >= si.first[j + 1]) ++j;
        const int64_t lo = (int64_t)si.bound[j] + (int64_t)(c - si.first[j]) * ((int64_t)CH << j);
        int64_t hi = lo + ((int64_t)CH << j);
        if (hi > (int64_t)si.bound[j + 1]) hi = si.bound[j + 1];
        const NormRec *nr = a.norm + s;
        const int valid = nr->valid;
        const __amdgpu_buffer_rsrc_t rsrc =
            make_rsrc((const char *)a.x + si.off * eb, (uint32_t)(si.len * eb));
        for (int64_t p0 = lo; p0 < hi; p0 += CH)
            walk_pass<HMAX, GREEDY, F16, F>(a, s, si, p0, hi, rsrc, nr->t, valid, st);
        if (threadIdx.x == 0) s_ticket = next;
        __syncthreads();
        t = s_ticket;
    }
    if (a.cand) stage_flush(st, a);
}

template <int HMAX, bool GREEDY, bool F16>
const void *kernel_ptr(int F) {
    switch (F) {
        case 1: return (const void *)k_sum_xcd<HMAX, GREEDY, F16, 1>;
        case 2: return (const void *)k_sum_xcd<HMAX, GREEDY, F16, 2>;
        default: return (const void *)k_sum_xcd<HMAX, GREEDY, F16, 4>;
    }
}

template <int HMAX>
const void *kernel_ptr_h(bool greedy, bool f16, int F) {
    if (greedy) return f16 ? kernel_ptr<HMAX, true, true>(F) : kernel_ptr<HMAX, true, false>(F);
    return f16 ? kernel_ptr<HMAX, false, true>(F) : kernel_ptr<HMAX, false, false>(F);
}

const void *xcd_kernel(int hmax, bool greedy, bool f16, int F) {
    switch (hmax) {
        case 4: return kernel_ptr_h<4>(greedy, f16, F);
        case 8: return kernel_ptr_h<8>(greedy, f16, F);
        case 16: return kernel_ptr_h<16>(greedy, f16, F);
        default: return kernel_ptr_h<32>(greedy, f16, F);
    }
}

}  // namespace

hipError_t xcd_resident_blocks(int hmax, bool greedy, bool f16, int F, int *per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, xcd_kernel(hmax, greedy, f16, F), kBlock, 0);
}

hipError_t launch_sum_xcd(const XcdArgs &a, int hmax, bool greedy, bool f16, int F, int blocks, hipStream_t st) {
    void *args[] = {(void *)&a};
    return hipLaunchKernel(xcd_kernel(hmax, greedy, f16, F), dim3(blocks), dim3(kBlock), args, 0, st);
}

}  // namespace hs
