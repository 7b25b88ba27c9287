// Ray-tiled harmonic sum over an f-fdot plane (gfx950).
//
// Harmonic k of fundamental (z, r) is the element (k z, k r) (+ drift along
// r), so every element a fundamental reads lies on its own ray through the
// origin, and two fundamentals share elements only if they lie on the same
// ray.  Grouping fundamentals by ray therefore closes the access pattern: a
// tile is a range of ratios [r0, r0 + delta) of one side (z > 0 or z < 0,
// rows u = |z|), holding the fundamentals u r0 <= r < u (r0 + delta) of
// every row u, and its harmonics read row m = k u only inside columns
// [m r0, m (r0 + delta)] (the greedy pair ends at k r + k <= m (r0 + delta)).
// Each tile stages that window of rows u_lo..b once from HBM into LDS
// (coalesced row segments), then walks all of its fundamentals out of LDS,
// so the plane is read about once instead of once per (row, harmonic) pair.
// The windows of the tiles of a side partition its rows; the tile width
// grows as fewer rows reach the ratio range (bands of equal top row b) so
// that every window fits the LDS budget.  Row z = 0 reads only itself (all
// of its fundamentals share one ray) and runs as a plain 1-row launch.
//
// The arithmetic of a fundamental is the same as in the plain plane kernel
// (float sum in harmonic order, fmaf normalisation, strict comparisons), so
// the outputs are identical bit for bit.
#include "hs_internal.h"

namespace hs {
namespace {

// LDS position of window element g: one pad word per 32 elements so that the
// stride-k reads of a wave (k a power of two) spread over the banks.
__device__ __forceinline__ int lds_pos(int g) { return g + (g >> 5); }

__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Band table: one thread per band, block-wide exclusive scan of tile counts.
__global__ __launch_bounds__(kRayMaxBands) void k_ray_bands(RayGeom g, RayBand *bands) {
    __shared__ uint32_t scan[kRayMaxBands];
    const int t = threadIdx.x;
    const int nb0 = ray_side_bands(g, 0), nb = nb0 + ray_side_bands(g, 1);
    RayBand rec{};
    uint32_t tiles = 0;
    if (t < nb) {
        rec.side = t < nb0 ? 0 : 1;
        const int j = t < nb0 ? t : t - nb0;
        rec.b = g.u_hi[rec.side] - j;
        tiles = ray_band(g, rec.side, j, &rec.start, &rec.end, &rec.delta);
    }
    scan[t] = tiles;
    __syncthreads();
    for (int o = 1; o < kRayMaxBands; o <<= 1) {
        const uint32_t v = t >= o ? scan[t - o] : 0u;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    if (t < nb) {
        rec.first_tile = scan[t] - tiles;
        bands[t] = rec;
    }
}

constexpr int kLoadBatch = 8;   // window loads in flight per thread

// Constants of row u = |z| in a tile: harmonics inside the plane (kq), the
// column threshold above which fewer fit, the window offsets of harmonic 1
// and their first and second differences, the first column and the output
// row offset.
struct RowRec {
    int32_t kq, kthr, T1, D1, E, rbase;
    int64_t rowoff;
};
constexpr int kRayStage = 64;   // candidate records staged per wave

// Window element: the stored power (simple sum) or the pair (x[c], x[c+1])
// that a greedy step compares (one 8-byte LDS read per step).
template <bool GREEDY>
struct WinT {
    using type = float;
};
template <>
struct WinT<true> {
    using type = float2;
};

template <int HMAX, bool GREEDY, bool F16>
__global__ __launch_bounds__(kBlock) void k_sum_2d_ray(Ray2dArgs a) {
    using W = typename WinT<GREEDY>::type;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    W *win = reinterpret_cast<W *>(lds_raw);
    __shared__ int64_t s_r0, s_r1;
    __shared__ int32_t s_side, s_b;
    __shared__ float2 s_tab[HMAX];
    __shared__ RowRec s_rows[kRayMaxRows];

    const uint32_t t = (blockIdx.x % (uint32_t)a.n_xcd) * a.per_xcd + blockIdx.x / (uint32_t)a.n_xcd;
    if (t >= a.n_tiles) return;   // uniform over the block
    // the tile's band: the one band j with first_tile(j) <= t < first_tile(j + 1)
    // (bands without tiles never match), found by all threads in parallel; the
    // float table goes to LDS (one global read per entry per tile)
    for (int j = threadIdx.x; j < a.n_bands; j += kBlock) {
        const RayBand bd = a.bands[j];
        if (bd.first_tile <= t && (j + 1 == a.n_bands || a.bands[j + 1].first_tile > t)) {
            const int64_t r0 = bd.start + (int64_t)(t - bd.first_tile) * bd.delta;
            s_r0 = r0;
            s_r1 = r0 + bd.delta < bd.end ? r0 + bd.delta : bd.end;
            s_side = bd.side;
            s_b = bd.b;
        }
    }
    if (threadIdx.x < HMAX) s_tab[threadIdx.x] = a.s.norm->t[threadIdx.x];
    __syncthreads();
    const int32_t r0 = uni((int32_t)s_r0);            // b r0 <= n_r - 1 < 2^30
    const int32_t dt = uni((int32_t)(s_r1 - s_r0));
    const int32_t side = uni(s_side), b = uni(s_b);
    const int32_t u_lo = a.g.u_lo[side], u_hi = a.g.u_hi[side];
    const int32_t sgn = side ? -1 : 1;
    const int32_t n_r = (int32_t)a.s.n_r;
    const int32_t c0 = u_lo * (u_lo - 1) / 2;
    const int lane = (int)(threadIdx.x & 63);
    // logical window offset of row m (rows and offsets are small: 24-bit products)
    auto row_base = [&](int32_t m) -> int32_t {
        return __umul24((uint32_t)dt, (uint32_t)((__umul24((uint32_t)m, (uint32_t)(m - 1)) >> 1) - c0)) + (m - u_lo);
    };

    // per-row constants of the fundamentals' walk (rows u_lo..b)
    for (int32_t i = threadIdx.x; i <= b - u_lo; i += kBlock) {
        const int32_t u = u_lo + i;
        RowRec rr;
        rr.kq = u_hi / u < a.s.H ? u_hi / u : a.s.H;   // harmonics inside the plane
        rr.kthr = (n_r - 1) / rr.kq;                   // den > kthr <=> fewer than kq harmonics fit
        rr.T1 = row_base(u);
        rr.E = __umul24((uint32_t)dt, (uint32_t)(u * u));
        rr.D1 = rr.E + __umul24((uint32_t)dt, (uint32_t)(u * (u - 1) / 2)) + u;
        rr.rbase = u * r0;
        rr.rowoff = ((int64_t)sgn * u - a.s.z_min) * (int64_t)n_r;
        s_rows[i] = rr;
    }

    // 1. window: rows u_lo..b, row m = m dt + 1 logical columns from m r0
    //    (loaded up to n_r - 1); each wave walks its rows u_lo + w, + 4, ...
    //    in 64-column chunks and issues kLoadBatch chunks before storing
    {
        int32_t m = u_lo + (int32_t)(threadIdx.x >> 6), c = 0;   // wave-uniform cursor
        while (m <= b) {
            W v[kLoadBatch];
            int32_t pos[kLoadBatch];
#pragma unroll
            for (int j = 0; j < kLoadBatch; ++j) {
                pos[j] = -1;
                if (m <= b) {
                    const int32_t col0 = m * r0;               // <= n_r - 1 for m <= b
                    const int32_t avail = n_r - col0;          // columns left in the row
                    const int32_t col = c + lane;
                    if (col <= m * dt && col < avail) {
                        const char *row = (const char *)a.s.plane +
                                          ((int64_t)sgn * m - a.s.z_min) * a.s.stride * (int64_t)(F16 ? 2 : 4);
                        float x0, x1 = 0.0f;
                        if constexpr (F16) {
                            const uint16_t *h = (const uint16_t *)row + col0 + col;
                            x0 = (float)__builtin_bit_cast(_Float16, h[0]);
                            if (GREEDY && col + 1 < avail) x1 = (float)__builtin_bit_cast(_Float16, h[1]);
                        } else {
                            const float *f = (const float *)row + col0 + col;
                            x0 = f[0];
                            if (GREEDY && col + 1 < avail) x1 = f[1];
                        }
                        if constexpr (GREEDY)
                            v[j] = make_float2(x0, x1);
                        else
                            v[j] = x0;
                        pos[j] = lds_pos(row_base(m) + col);
                    }
                    c += 64;
                    if (c > m * dt) {
                        m += kBlock / 64;
                        c = 0;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kLoadBatch; ++j)
                if (pos[j] >= 0) win[pos[j]] = v[j];
        }
    }
    __syncthreads();

    // 2. fundamentals, flat order (row u_lo first, columns within a row):
    //    wave w owns a contiguous quarter, lane l takes positions l, l + 64,
    //    ... of it, so each lane's (row u, column offset R) advances by 64
    //    per iteration and rows are crossed incrementally.  Per row the lane
    //    keeps the window offset of harmonic k's row, T_k = base(k u), as a
    //    second-order difference (T_{k+1} = T_k + D_k, D_{k+1} = D_k + dt u^2).
    //    Candidates are staged per wave behind the window.
    Stage st{(hs_candidate *)(lds_raw + ray_window_bytes(a.g.budget, GREEDY)) + (threadIdx.x >> 6) * kRayStage, 0};
    const int valid = a.s.norm->valid;
    const int32_t n_end = a.s.n_end < (int64_t)n_r ? (int32_t)a.s.n_end : n_r;
    const int32_t nr1 = n_r - 1;
    const int32_t nf = __umul24((uint32_t)dt, (uint32_t)(b * (b + 1) / 2 - c0));
    const int32_t wq = (nf + kBlock - 1) / kBlock * 64;   // per wave: ceil(nf / 4) rounded up to 64
    const int32_t fw0 = (int32_t)(threadIdx.x >> 6) * wq;
    const int32_t fw1 = fw0 + wq < nf ? fw0 + wq : nf;
    int32_t u = u_lo, R = 0;
    if (fw0 + lane < nf) {
        // row of flat position f: the smallest u with tri(u) > f / dt + c0
        const int32_t f = fw0 + lane;
        const int32_t y = (int32_t)((float)f / (float)dt) + c0;   // exact: f, dt < 2^24
        u = (int32_t)((__builtin_sqrtf(8.0f * (float)y + 1.0f) - 1.0f) * 0.5f) + 1;
        while (u * (u + 1) / 2 <= y) ++u;
        while (u * (u - 1) / 2 > y) --u;
        R = f - __umul24((uint32_t)dt, (uint32_t)(u * (u - 1) / 2 - c0));
    }
    // per-row state of the lane
    int32_t rowlen = u * dt;
    RowRec rw = s_rows[u - u_lo];
    for (int32_t f0 = fw0; f0 < fw1; f0 += 64) {   // wave-uniform trip count
        const int32_t r = rw.rbase + R;
        const bool in = f0 + lane < fw1 && r < n_r;
        int K = 0;
        if (in && valid && r >= a.s.first_bin && r < n_end) {
            const int32_t den = GREEDY ? r + 1 : r;
            K = rw.kq;
            if (den > rw.kthr) {   // exact quotient (< kq <= 32) from a float estimate
                int q = (int)((float)nr1 / (float)den);
                if ((int64_t)(q + 1) * den <= nr1) ++q;
                else if ((int64_t)q * den > nr1) --q;
                K = q;
            }
        }
        float S = 0.0f, best = -__builtin_inff();   // any finite SNR beats it: the first eligible k wins
        int kb = 0, db = 0;
        int32_t d = 0, T = rw.T1, D = rw.D1, kR = R;
#pragma unroll
        for (int k = 1; k <= HMAX; ++k) {
            if (k > K) break;
            const int32_t g = T + kR + d;
            float v;
            if constexpr (GREEDY) {
                const float2 p = win[lds_pos(g)];
                const bool up = p.y > p.x;
                v = up ? p.y : p.x;
                d += up ? 1 : 0;
            } else {
                v = win[lds_pos(g)];
            }
            S = S + v;
            const float2 tk = s_tab[k - 1];
            const float snr = __builtin_fmaf(S, tk.x, tk.y);
            if ((a.s.kmask >> (k - 1)) & 1ull) {
                if (snr > best) {
                    best = snr;
                    kb = k;
                    db = d;
                }
            }
            T += D;
            D += rw.E;
            kR += R;
        }
        const Best bs{kb ? best : 0.0f, kb, db};
        const int64_t o = rw.rowoff + r;
        if (in) {
            if (a.s.snr) a.s.snr[o] = bs.snr;
            if (a.s.harm) a.s.harm[o] = (uint8_t)bs.harm;
            if (a.s.drift) a.s.drift[o] = (uint8_t)bs.drift;
        }
        if (a.s.cand) {
            hs_candidate rec;
            rec.spectrum = 0u;
            rec.bin = (uint32_t)o;
            rec.snr = bs.snr;
            rec.harm = (uint16_t)bs.harm;
            rec.drift = (uint16_t)bs.drift;
            stage_push<kRayStage>(st, a.s.cand, a.s.cap, a.s.count, in && bs.harm > 0 && bs.snr > a.s.thr, rec);
        }
        R += 64;
        if (R >= rowlen && u < b) {
            do {
                R -= rowlen;
                ++u;
                rowlen += dt;
            } while (R >= rowlen && u < b);
            rw = s_rows[u - u_lo];
        }
    }
    if (a.s.cand) stage_flush(st, a.s.cand, a.s.cap, a.s.count);
}

template <int HMAX>
hipError_t ray_h(const Ray2dArgs &a, bool greedy, bool f16, dim3 grid, size_t lds, hipStream_t st) {
    if (greedy) {
        if (f16)
            hipLaunchKernelGGL((k_sum_2d_ray<HMAX, true, true>), grid, dim3(kBlock), lds, st, a);
        else
            hipLaunchKernelGGL((k_sum_2d_ray<HMAX, true, false>), grid, dim3(kBlock), lds, st, a);
    } else {
        if (f16)
            hipLaunchKernelGGL((k_sum_2d_ray<HMAX, false, true>), grid, dim3(kBlock), lds, st, a);
        else
            hipLaunchKernelGGL((k_sum_2d_ray<HMAX, false, false>), grid, dim3(kBlock), lds, st, a);
    }
    return hipGetLastError();
}

}  // namespace

// Bands, then the tiles of both sides.  The caller checked ray_feasible and
// launches row z = 0 separately.
hipError_t launch_sum_2d_ray(Ray2dArgs a, int hmax, bool greedy, bool f16, hipStream_t st) {
    a.n_bands = ray_side_bands(a.g, 0) + ray_side_bands(a.g, 1);
    uint32_t tiles = 0;
    for (int side = 0; side < 2; ++side)
        for (int j = 0; j < ray_side_bands(a.g, side); ++j) {
            int64_t s, e;
            int32_t d;
            tiles += ray_band(a.g, side, j, &s, &e, &d);
        }
    if (a.n_bands == 0 || tiles == 0) return hipSuccess;
    a.n_tiles = tiles;
    if (a.n_xcd < 1) a.n_xcd = 1;
    a.per_xcd = (tiles + (uint32_t)a.n_xcd - 1) / (uint32_t)a.n_xcd;
    hipLaunchKernelGGL(k_ray_bands, dim3(1), dim3(kRayMaxBands), 0, st, a.g, a.bands);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(a.per_xcd * (uint32_t)a.n_xcd);
    const size_t lds = ray_window_bytes(a.g.budget, greedy) +
                       (a.s.cand ? sizeof(hs_candidate) * (kBlock / 64) * kRayStage : 0);
    switch (hmax) {
        case 4: return ray_h<4>(a, greedy, f16, grid, lds, st);
        case 8: return ray_h<8>(a, greedy, f16, grid, lds, st);
        case 16: return ray_h<16>(a, greedy, f16, grid, lds, st);
        case 32: return ray_h<32>(a, greedy, f16, grid, lds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hs
