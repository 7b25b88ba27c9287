// Persistent, XCD-aware harmonic-sum kernel (gfx950) for one spectrum or a
// batch of spectra of any lengths.
//
// Why: a fundamental's k-th harmonic reads bins near k n, so over all
// fundamentals and harmonics every cache line of a spectrum is touched about
// once per harmonic (N H s bytes for N bins of s bytes).  Whether those
// touches hit the XCD's 4 MB L2 or go to the Infinity Fabric depends only on
// scheduling: when the resident workgroups of one XCD work on a narrow band of
// consecutive fundamentals, the windows [k a, k (a + D)] of neighbouring
// harmonics overlap and stay in that XCD's L2.
//
// How: every spectrum's fundamentals are cut into chunks of roughly equal
// work (chunk size grows as the number of harmonics that fit shrinks, see
// spec_info) and the chunks of all spectra are concatenated in order.  The
// grid holds as many workgroups as can be resident; workgroup b serves work
// queue b % n_xcd (the hardware dispatches workgroups to XCDs round robin;
// correctness does not depend on it), and queue q owns the q-th of n_xcd equal
// contiguous slices of the chunk list, handed out in order through one atomic
// ticket counter.  So each XCD sweeps its own slice front to back with its
// resident workgroups on adjacent chunks.  A ticket beyond the slice ends the
// workgroup: every wave reaches the exit.
//
// Per lane: F fundamentals (p0 + threadIdx.x + f kBlock) walked harmonic by
// harmonic with independent loads in flight.  When every fundamental of the
// wave sums the same number of harmonics K, all eligible (almost every
// wave), the walk has no per-lane bound (walk_uniform).  Otherwise the loop
// bound is the wave's largest K and a lane whose own K is smaller issues its
// loads at an out-of-range buffer offset, which returns zero without
// touching memory, and commits nothing (walk_lanes).
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

__device__ __forceinline__ void spec_info(SpecInfo &r, const int64_t *offsets, int64_t n_bins, int s, uint32_t base,
                                          int H) {
    if (offsets) {
        r.off = offsets[s];
        r.len = offsets[s + 1] - r.off;
    } else {                                            // one spectrum of n_bins
        r.off = 0;
        r.len = n_bins;
    }
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

// Candidate staging (Stage in hs_device.h): each wave collects its records in
// its own LDS slice of kStage records and reserves space in the global list
// with one atomic per flush (a device-wide atomic per record would serialise
// the whole kernel on one address).
constexpr int kStage = 256;

// Harmonic walk of a pass with a bound per lane: each lane sums its own
// K = min(H, (len - 1) / (n + greedy)) harmonics (0 outside [first_bin,
// n_end)); the loop runs to the wave's largest K, lanes past their own K
// load at an out-of-range offset (zero, no memory access) and commit nothing.
template <int HMAX, bool GREEDY, bool F16, int F>
__device__ __forceinline__ void walk_lanes(const SumArgs &a, int64_t len, int64_t n_end, int64_t p0, int wave,
                                           __amdgpu_buffer_rsrc_t rsrc, const float2 *tab, int valid,
                                           const uint32_t (&n)[F], float (&bs)[F], int (&kbo)[F], int (&dbo)[F]) {
    using L = Loader<F16>;
    constexpr uint32_t eb = L::kBytes;
    int K[F];
    uint32_t m[F], d[F];
    float S[F], best[F];
    int kb[F], db[F];
    int KW = 0;                                             // wave-uniform loop bound
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int64_t n0 = p0 + f * kBlock;                 // first fundamental of this f-slice
        K[f] = valid ? keff<GREEDY>(n0 + threadIdx.x, len, a.first_bin, n_end, a.H) : 0;
        // K is non-increasing in n: the wave's largest K is at its first fundamental >= first_bin
        int64_t nw = n0 + (int64_t)wave * 64;
        if (nw < a.first_bin) nw = a.first_bin;
        const int kw = valid ? keff<GREEDY>(nw, len, a.first_bin, n_end, a.H) : 0;
        KW = kw > KW ? kw : KW;
        KW = __builtin_amdgcn_readfirstlane(KW);           // wave-uniform by construction
        m[f] = n[f];
        d[f] = 0;
        S[f] = 0.0f;
        best[f] = 0.0f;                                    // no eligible k yet (kb == 0)
        kb[f] = 0;
        db[f] = 0;
    }
#pragma unroll
    for (int k = 1; k <= HMAX; ++k) {
        if (k > KW) continue;                               // wave-uniform: skips the rest
        const float2 tk = tab[k - 1];
        const bool el = (a.kmask >> (k - 1)) & 1ull;
        if constexpr (F16) {
            // 16-bit storage: issue the loads of every slice first, so that F
            // independent loads of the wave are in flight together, then
            // consume them in order (the eligibility test is folded into the
            // update mask: no branch between); 5.75 against 7.56 ms on the
            // 512-spectrum batch at F = 4, where the fused loop below kept one
            // load in flight per wave.  For FP32 the fused loop measured faster
            // (11.2 against 11.6-11.7 ms): that walk is bound by traffic fetched
            // beyond the L2, and more loads in flight only add to it.
            uint32_t w32[F];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const bool act = k <= K[f];
                if constexpr (GREEDY) {   // both halves with one 4-byte load (2-byte aligned for odd pairs)
                    const uint32_t o = act ? (m[f] + d[f]) * eb : kOob;
                    w32[f] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)o, 0, 0);
                } else {
                    const uint32_t o = act ? m[f] * eb : kOob;
                    w32[f] = __builtin_amdgcn_raw_buffer_load_b16(rsrc, (int)o, 0, 0);
                }
            }
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const bool act = k <= K[f];
                float v;
                if constexpr (GREEDY) {
                    const float2 p = make_float2((float)__builtin_bit_cast(_Float16, (unsigned short)(w32[f] & 0xFFFFu)),
                                                 (float)__builtin_bit_cast(_Float16, (unsigned short)(w32[f] >> 16)));
                    const bool up = p.y > p.x;              // inactive lanes read (0, 0): no move
                    v = up ? p.y : p.x;
                    d[f] += up ? 1u : 0u;
                } else {
                    v = (float)__builtin_bit_cast(_Float16, (unsigned short)(w32[f] & 0xFFFFu));
                }
                S[f] = S[f] + v;                            // + 0 on inactive lanes
                const float snr = __builtin_fmaf(S[f], tk.x, tk.y);
                // eligible k only (el is wave-uniform); the first eligible k, then strict >
                const bool upd = el && act && (kb[f] == 0 || snr > best[f]);
                best[f] = upd ? snr : best[f];
                kb[f] = upd ? k : kb[f];
                db[f] = upd ? (int)d[f] : db[f];
                m[f] += n[f];
            }
        } else {
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const bool act = k <= K[f];
                float v;
                if constexpr (GREEDY) {
                    const uint32_t o = act ? (m[f] + d[f]) * eb : kOob;
                    const f32x2_t w =
                        __builtin_bit_cast(f32x2_t, __builtin_amdgcn_raw_buffer_load_b64(rsrc, (int)o, 0, 0));
                    const bool up = w.y > w.x;              // inactive lanes read (0, 0): no move
                    v = up ? w.y : w.x;
                    d[f] += up ? 1u : 0u;
                } else {
                    const uint32_t o = act ? m[f] * eb : kOob;
                    v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)o, 0, 0));
                }
                S[f] = S[f] + v;                            // + 0 on inactive lanes
                if (el) {                                   // wave-uniform
                    const float snr = __builtin_fmaf(S[f], tk.x, tk.y);
                    const bool upd = act && (kb[f] == 0 || snr > best[f]);   // the first eligible k, then strict >
                    best[f] = upd ? snr : best[f];
                    kb[f] = upd ? k : kb[f];
                    db[f] = upd ? (int)d[f] : db[f];
                }
                m[f] += n[f];
            }
        }
    }
#pragma unroll
    for (int f = 0; f < F; ++f) {
        bs[f] = kb[f] ? best[f] : 0.0f;
        kbo[f] = kb[f];
        dbo[f] = db[f];
    }
}

// Harmonic walk of a pass in which every lane of the wave, in all F slices,
// is a fundamental with the same harmonic count KU and every k <= KU is
// eligible (the common case: K changes only near len / k, and a wave holds
// 64 consecutive fundamentals).  No bound or eligibility test per lane is
// needed: every step loads, selects and updates.  The greedy walk keeps one
// index per fundamental, md = k n + d (the left element of harmonic k's
// pair), advanced by n + up; the drift at the best harmonic comes from the
// index after that step, d = md' - (kb + 1) n.  Same sums, same SNRs, same
// comparisons as the walk with a bound per lane.
template <int HMAX, bool GREEDY, bool F16, int F>
__device__ __forceinline__ void walk_uniform(int KU, __amdgpu_buffer_rsrc_t rsrc, const float2 *tab,
                                             const uint32_t (&n)[F], float (&bs)[F], int (&kbo)[F], int (&dbo)[F]) {
    constexpr uint32_t eb = Loader<F16>::kBytes;
    uint32_t md[F], mdb[F];
    float S[F], best[F];
    int kb[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
        md[f] = n[f];
        mdb[f] = 0;
        S[f] = 0.0f;
        best[f] = 0.0f;
        kb[f] = 0;
    }
#pragma unroll
    for (int k = 1; k <= HMAX; ++k) {
        if (k > KU) break;                                  // wave-uniform
        const float2 tk = tab[k - 1];
        float v[F];
        uint32_t nx[F];
        if constexpr (F16) {
            // all slices' loads first, then their use (F loads of the wave in flight)
            uint32_t w[F];
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if constexpr (GREEDY)   // both halves with one 4-byte load
                    w[f] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(md[f] * eb), 0, 0);
                else
                    w[f] = __builtin_amdgcn_raw_buffer_load_b16(rsrc, (int)(md[f] * eb), 0, 0);
            }
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const float x0 = (float)__builtin_bit_cast(_Float16, (unsigned short)(w[f] & 0xFFFFu));
                if constexpr (GREEDY) {
                    const float x1 = (float)__builtin_bit_cast(_Float16, (unsigned short)(w[f] >> 16));
                    const bool up = x1 > x0;
                    v[f] = up ? x1 : x0;
                    nx[f] = md[f] + n[f] + (up ? 1u : 0u);
                } else {
                    v[f] = x0;
                    nx[f] = md[f] + n[f];
                }
            }
        } else {
#pragma unroll
            for (int f = 0; f < F; ++f) {
                if constexpr (GREEDY) {
                    const f32x2_t p =
                        __builtin_bit_cast(f32x2_t, __builtin_amdgcn_raw_buffer_load_b64(rsrc, (int)(md[f] * eb), 0, 0));
                    const bool up = p.y > p.x;
                    v[f] = up ? p.y : p.x;
                    nx[f] = md[f] + n[f] + (up ? 1u : 0u);
                } else {
                    v[f] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(md[f] * eb), 0, 0));
                    nx[f] = md[f] + n[f];
                }
            }
        }
#pragma unroll
        for (int f = 0; f < F; ++f) {
            S[f] = S[f] + v[f];
            const float snr = __builtin_fmaf(S[f], tk.x, tk.y);
            const bool upd = k == 1 || snr > best[f];      // the first eligible k, then strict >
            best[f] = upd ? snr : best[f];
            kb[f] = upd ? k : kb[f];
            if constexpr (GREEDY) mdb[f] = upd ? nx[f] : mdb[f];
            md[f] = nx[f];
        }
    }
#pragma unroll
    for (int f = 0; f < F; ++f) {
        bs[f] = kb[f] ? best[f] : 0.0f;
        kbo[f] = kb[f];
        dbo[f] = (GREEDY && kb[f]) ? (int)(mdb[f] - (uint32_t)(kb[f] + 1) * n[f]) : 0;
    }
}

// One pass: kBlock * F consecutive fundamentals starting at p0 (lane owns
// p0 + f kBlock + threadIdx.x), restricted to [p0, p_end).  The wave takes
// the uniform walk when its first and last fundamental (K is non-increasing
// in n) have the same harmonic count, it holds no bin outside [first_bin,
// n_end) and the eligibility mask covers harmonics 1..K (uniform_k, from
// the spectrum's thresholds); else the walk with a bound per lane.
template <int HMAX, bool GREEDY, bool F16, int F>
__device__ __forceinline__ void walk_pass(const SumArgs &a, int s, const SpecInfo &si, int64_t p0, int64_t p_end,
                                          __amdgpu_buffer_rsrc_t rsrc, const float2 *tab, int valid,
                                          int32_t thr, Stage &st) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t len = si.len;
    int64_t n_end = a.n_end < len ? a.n_end : len;
    if (p_end < n_end) n_end = p_end;
    uint32_t n[F];
#pragma unroll
    for (int f = 0; f < F; ++f) n[f] = (uint32_t)(p0 + f * kBlock + threadIdx.x);
    const int64_t wf = p0 + (int64_t)wave * 64, wl = wf + (F - 1) * kBlock + 63;
    const int KU = valid ? uniform_k(thr, wf, wl, a.first_bin, n_end, a.kmask) : 0;
    float bs[F];
    int kb[F], db[F];
    if (KU > 0)
        walk_uniform<HMAX, GREEDY, F16, F>(KU, rsrc, tab, n, bs, kb, db);
    else
        walk_lanes<HMAX, GREEDY, F16, F>(a, len, n_end, p0, wave, rsrc, tab, valid, n, bs, kb, db);
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const bool in = (int64_t)n[f] < p_end;
        if (in) {   // outputs are never read again: non-temporal stores
            const int64_t o = si.off + n[f];
            if (a.snr) __builtin_nontemporal_store(bs[f], a.snr + o);
            if (a.harm) __builtin_nontemporal_store((uint8_t)kb[f], a.harm + o);
            if (a.drift) __builtin_nontemporal_store((uint8_t)db[f], a.drift + o);
        }
        if (a.cand) {
            hs_candidate r;
            r.spectrum = (uint32_t)s;
            r.bin = n[f];
            r.snr = bs[f];
            r.harm = (uint16_t)kb[f];
            r.drift = (uint16_t)db[f];
            stage_push<kStage>(st, a.cand, a.cap, a.count, in && kb[f] > 0 && bs[f] > a.thr, r);
        }
    }
}

// Exclusive prefix of the chunk counts of all spectra (one block).
__global__ __launch_bounds__(1024) void k_chunk_prefix(const int64_t *offsets, int64_t n_bins, int n_spectra, int H,
                                                      uint32_t chunk, uint32_t *prefix) {
    __shared__ uint32_t carry;
    __shared__ uint32_t part[1024];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < n_spectra; b0 += 1024) {
        const int s = b0 + threadIdx.x;
        uint32_t c = 0;
        if (s < n_spectra) {
            SpecInfo si;
            spec_info(si, offsets, n_bins, s, chunk, H);
            c = si.chunks;
        }
        part[threadIdx.x] = c;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {               // inclusive scan
            uint32_t v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0u;
            __syncthreads();
            part[threadIdx.x] += v;
            __syncthreads();
        }
        if (s < n_spectra) prefix[s] = carry + part[threadIdx.x] - c;
        __syncthreads();
        if (threadIdx.x == 0) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) prefix[n_spectra] = carry;
}

// Occupancy: up to 8 waves per SIMD (8 workgroups of 256 per CU).  The
// walks need 35-80 VGPRs at every H bucket and F with no scratch, so 6-7
// workgroups fit per CU; the launch-shape tuner picks how many run.
template <int HMAX, bool GREEDY, bool F16, int F>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 8))) void k_sum_xcd(XcdArgs xa) {
    constexpr uint32_t eb = Loader<F16>::kBytes;
    constexpr int CH = kBlock * F;                 // fundamentals per pass (class-0 chunk)
    const SumArgs &a = xa.s;
    const int q = blockIdx.x % xa.n_xcd;
    __shared__ uint32_t s_ticket;
    __shared__ hs_candidate s_stage[kBlock / 64][kStage];
    __shared__ float2 s_tab[HS_MAX_HARMONICS];     // (rs_k, nm_k) of the current spectrum
    Stage st{s_stage[threadIdx.x >> 6], 0};
    int tab_s = -1;                                 // spectrum whose table is in s_tab
    int thr_s = -1;                                 // spectrum whose harmonic-count thresholds are in thr
    int32_t thr = -1;

    // this queue's slice [g0, g1) of the concatenated chunk list
    const uint32_t total = xa.prefix[xa.n_spectra];
    const uint32_t g0 = (uint32_t)((uint64_t)total * q / xa.n_xcd);
    const uint32_t g1 = (uint32_t)((uint64_t)total * (q + 1) / xa.n_xcd);
    // spectrum holding chunk g0: last s with prefix[s] <= g0 (binary search, uniform)
    int s = 0;
    {
        int lo = 0, hi = xa.n_spectra - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (xa.prefix[mid] <= g0) lo = mid; else hi = mid - 1;
        }
        s = lo;
    }
    SpecInfo si;
    spec_info(si, a.offsets, a.n_bins, s, CH, a.H);
    uint32_t base = xa.prefix[s];                  // global index of spectrum s's first chunk

    if (threadIdx.x == 0) s_ticket = atomicAdd(xa.tickets + q, 1u);
    __syncthreads();
    // readfirstlane: the ticket is block-uniform; making that visible to the
    // compiler keeps everything derived from it (spectrum, chunk, table
    // address) in SGPRs and the table reads scalar
    uint32_t t = __builtin_amdgcn_readfirstlane(s_ticket);
    for (;;) {
        __syncthreads();                            // everyone has read s_ticket
        uint32_t next = 0;
        if (threadIdx.x == 0) next = atomicAdd(xa.tickets + q, 1u);   // prefetch: used after this chunk
        const uint32_t g = g0 + t;
        if (g >= g1) break;                                    // slice exhausted (uniform)
        while (g >= base + si.chunks) {                        // advance to the spectrum holding g
            base += si.chunks;
            ++s;
            spec_info(si, a.offsets, a.n_bins, s, CH, a.H);
        }
        const uint32_t c = g - base;
        // class of chunk c: the last class whose first chunk is <= c (unrolled
        // with constant indices, so the tables stay in registers)
        int j = 0;
        uint32_t fj = si.first[0], bj = si.bound[0], bj1 = si.bound[1];
#pragma unroll
        for (int i = 1; i < kClasses; ++i)
            if (c >= si.first[i]) {
                j = i;
                fj = si.first[i];
                bj = si.bound[i];
                bj1 = si.bound[i + 1];
            }
        const int64_t lo = (int64_t)bj + (int64_t)(c - fj) * ((int64_t)CH << j);
        int64_t hi = lo + ((int64_t)CH << j);
        if (hi > (int64_t)bj1) hi = bj1;
        const NormRec *nr = a.norm + __builtin_amdgcn_readfirstlane(s);
        const int valid = nr->valid;
        if (s != tab_s) {                                      // uniform: reload the table
            if (threadIdx.x < HS_MAX_HARMONICS) s_tab[threadIdx.x] = nr->t[threadIdx.x];
            __syncthreads();
            tab_s = s;
        }
        const __amdgpu_buffer_rsrc_t rsrc =
            make_rsrc((const char *)a.x + si.off * eb, (uint32_t)(si.len * eb));
        if (s != thr_s) {                                      // uniform: thresholds of spectrum s
            thr = k_threshold<GREEDY>(si.len, a.H);
            thr_s = s;
        }
        for (int64_t p0 = lo; p0 < hi; p0 += CH)
            walk_pass<HMAX, GREEDY, F16, F>(a, s, si, p0, hi, rsrc, s_tab, valid, thr, st);
        if (threadIdx.x == 0) s_ticket = next;
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_ticket);
    }
    if (a.cand) stage_flush(st, a.cand, a.cap, a.count);
}

template <int HMAX, bool GREEDY, bool F16>
const void *kernel_ptr(int F) {
    if (F == 1) return (const void *)k_sum_xcd<HMAX, GREEDY, F16, 1>;
    return F == 2 ? (const void *)k_sum_xcd<HMAX, GREEDY, F16, 2> : (const void *)k_sum_xcd<HMAX, GREEDY, F16, 4>;
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
        case 32: return kernel_ptr_h<32>(greedy, f16, F);
        default: return kernel_ptr_h<64>(greedy, f16, F);
    }
}

}  // namespace

hipError_t xcd_resident_blocks(int hmax, bool greedy, bool f16, int F, int *per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, xcd_kernel(hmax, greedy, f16, F), kBlock, 0);
}

hipError_t launch_sum_xcd(const XcdArgs &a, int hmax, bool greedy, bool f16, int F, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_chunk_prefix, dim3(1), dim3(1024), 0, st, a.s.offsets, a.s.n_bins, a.n_spectra, a.s.H,
                       (uint32_t)(kBlock * F), a.prefix);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&a};
    return hipLaunchKernel(xcd_kernel(hmax, greedy, f16, F), dim3(blocks), dim3(kBlock), args, 0, st);
}

}  // namespace hs
