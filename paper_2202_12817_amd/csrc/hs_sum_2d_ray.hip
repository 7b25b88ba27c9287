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

// Constants of row u = |z| in a tile: harmonics inside the plane (kq), the
// column threshold above which fewer fit, the window offsets of harmonic 1
// and their first and second differences, the first column and the output
// row offset.
struct RowRec {
    int32_t kq, kthr, T1, D1, E, rbase;
    int64_t rowoff;
};
constexpr int kRayStage = 64;   // candidate records staged per wave

struct Tile {
    int32_t side, b, r0, dt;
};

// Tile t from the band table; j is the band cursor (tiles only move forward).
__device__ __forceinline__ Tile tile_at(const Ray2dArgs &a, uint32_t t, int &j) {
    while (j + 1 < a.n_bands && a.bands[j + 1].first_tile <= t) ++j;
    const RayBand &bd = a.bands[j];
    const int64_t r0 = bd.start + (int64_t)(t - bd.first_tile) * bd.delta;
    const int64_t r1 = r0 + bd.delta < bd.end ? r0 + bd.delta : bd.end;
    Tile tl;
    tl.side = uni(bd.side);
    tl.b = uni(bd.b);
    tl.r0 = uni((int32_t)r0);   // b r0 <= n_r - 1 < 2^30
    tl.dt = uni((int32_t)(r1 - r0));
    return tl;
}

// Logical window offset of row m of a tile (24-bit products: rows and
// offsets are small).
__device__ __forceinline__ int32_t row_base(int32_t dt, int32_t c0, int32_t u_lo, int32_t m) {
    return __umul24((uint32_t)dt, (uint32_t)((__umul24((uint32_t)m, (uint32_t)(m - 1)) >> 1) - c0)) + (m - u_lo);
}

// This thread's share of a tile's window (elements g = threadIdx.x + 256 i
// of rows u_lo..b; row m holds m dt + 1 logical columns from m r0, read up
// to n_r - 1), loaded into registers: the loads stay in flight while the
// previous tile is walked.
template <bool F16>
__device__ __forceinline__ void window_load(const Ray2dArgs &a, const Tile &tl, float (&vals)[kRayMaxPer]) {
    const int32_t u_lo = a.g.u_lo[tl.side], b = tl.b, dt = tl.dt, r0 = tl.r0;
    const int32_t sgn = tl.side ? -1 : 1;
    const int32_t n_r = (int32_t)a.s.n_r;
    const int32_t c0 = u_lo * (u_lo - 1) / 2;
    const int32_t total = row_base(dt, c0, u_lo, b + 1);
    int32_t g = (int32_t)threadIdx.x;
    // row of g: the largest m with base(m) <= g (root of dt m (m - 1) / 2 + m = g + dt c0 + u_lo)
    const float fdt = (float)dt, hdt = 0.5f * fdt;
    int32_t m = (int32_t)(((hdt - 1.0f) +
                           __builtin_sqrtf((1.0f - hdt) * (1.0f - hdt) + 2.0f * fdt * (float)(g + dt * c0 + u_lo))) /
                          fdt);
    if (m < u_lo) m = u_lo;
    if (m > b) m = b;
    while (m < b && row_base(dt, c0, u_lo, m + 1) <= g) ++m;
    while (m > u_lo && row_base(dt, c0, u_lo, m) > g) --m;
    int32_t c = g - row_base(dt, c0, u_lo, m);
#pragma unroll
    for (int i = 0; i < kRayMaxPer; ++i) {
        vals[i] = 0.0f;
        if (g < total) {
            const int32_t col = m * r0 + c;
            if (col <= n_r - 1) {
                const int64_t e = ((int64_t)sgn * m - a.s.z_min) * a.s.stride + col;
                if constexpr (F16)
                    vals[i] = (float)__builtin_bit_cast(_Float16, ((const uint16_t *)a.s.plane)[e]);
                else
                    vals[i] = ((const float *)a.s.plane)[e];
            }
        }
        g += kBlock;
        c += kBlock;
        while (m <= b && c > m * dt) {
            c -= m * dt + 1;
            ++m;
        }
    }
}

// Walk every fundamental of a tile out of the staged window.
// Flat order (row u_lo first, columns within a row): wave w owns a
// contiguous quarter, lane l takes positions l, l + 64, ... of it, so each
// lane's (row u, column offset R) advances by 64 per iteration and rows are
// crossed incrementally.  Per row the lane keeps the window offset of
// harmonic k's row, T_k = base(k u), as a second-order difference
// (T_{k+1} = T_k + D_k, D_{k+1} = D_k + dt u^2).
template <int HMAX, bool GREEDY>
__device__ __forceinline__ void walk_tile(const Ray2dArgs &a, const Tile &tl, const float *win, const float2 *tab,
                                          const RowRec *rows, int valid, Stage &st) {
    const int32_t u_lo = a.g.u_lo[tl.side], b = tl.b, dt = tl.dt;
    const int32_t n_r = (int32_t)a.s.n_r;
    const int32_t c0 = u_lo * (u_lo - 1) / 2;
    const int32_t n_end = a.s.n_end < (int64_t)n_r ? (int32_t)a.s.n_end : n_r;
    const int32_t nr1 = n_r - 1;
    const int lane = (int)(threadIdx.x & 63);
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
    int32_t rowlen = u * dt;
    RowRec rw = rows[u - u_lo];
    for (int32_t f0 = fw0; f0 < fw1; f0 += 64) {   // wave-uniform trip count
        const int32_t r = rw.rbase + R;
        const bool in = f0 + lane < fw1 && r < n_r;
        int K = 0;
        if (in && valid && r >= a.s.first_bin && r < n_end) {
            const int32_t den = GREEDY ? r + 1 : r;
            K = rw.kq;
            if (den > rw.kthr) {   // exact quotient (< kq <= 32) from a float estimate
                int qv = (int)((float)nr1 / (float)den);
                if ((int64_t)(qv + 1) * den <= nr1) ++qv;
                else if ((int64_t)qv * den > nr1) --qv;
                K = qv;
            }
        }
        float S = 0.0f, best = 0.0f;                // kb == 0: no eligible k yet
        int kb = 0, db = 0;
        int32_t d = 0, T = rw.T1, D = rw.D1, kR = R;
#pragma unroll
        for (int k = 1; k <= HMAX; ++k) {
            if (k > K) break;
            const int32_t g = T + kR + d;
            float v;
            if constexpr (GREEDY) {
                const float x0 = win[lds_pos(g)], x1 = win[lds_pos(g + 1)];
                const bool up = x1 > x0;
                v = up ? x1 : x0;
                d += up ? 1 : 0;
            } else {
                v = win[lds_pos(g)];
            }
            S = S + v;
            const float2 tk = tab[k - 1];
            const float snr = __builtin_fmaf(S, tk.x, tk.y);
            if ((a.s.kmask >> (k - 1)) & 1ull) {
                if (kb == 0 || snr > best) {   // the first eligible k, then strict >
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
            rw = rows[u - u_lo];
        }
    }
}

// Persistent: XCD q (= blockIdx.x % n_xcd, the dispatcher's round robin)
// owns the tiles [T q / n_xcd, T (q + 1) / n_xcd) and its workgroups take
// them in turn, so adjacent tiles (adjacent output segments) run side by
// side on one XCD.  A workgroup stages tile i's window from registers into
// LDS, issues the loads of tile i + 1, then walks tile i.
template <int HMAX, bool GREEDY, bool F16>
__global__ __launch_bounds__(kBlock) void k_sum_2d_ray(Ray2dArgs a) {
    extern __shared__ __attribute__((aligned(16))) float win[];
    __shared__ float2 s_tab[HMAX];
    __shared__ RowRec s_rows[kRayMaxRows];

    const uint32_t nx = (uint32_t)a.n_xcd, q = blockIdx.x % nx, wi = blockIdx.x / nx, nw = gridDim.x / nx;
    const uint32_t xb = (uint32_t)((uint64_t)a.n_tiles * q / nx), xe = (uint32_t)((uint64_t)a.n_tiles * (q + 1) / nx);
    uint32_t t = xb + wi;
    if (t >= xe) return;   // uniform over the block
    if (threadIdx.x < HMAX) s_tab[threadIdx.x] = a.s.norm->t[threadIdx.x];
    const int valid = a.s.norm->valid;
    Stage st{(hs_candidate *)((unsigned char *)win + ray_window_bytes(a.g.budget, false)) +
                 (threadIdx.x >> 6) * kRayStage,
             0};
    int j = 0;
    {   // band of the first tile: the last band with first_tile <= t
        int lo = 0, hi = a.n_bands - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.bands[mid].first_tile <= t) lo = mid;
            else hi = mid - 1;
        }
        j = uni(lo);
    }
    Tile cur = tile_at(a, t, j);
    float vals[kRayMaxPer];
    window_load<F16>(a, cur, vals);
    for (;;) {
        __syncthreads();   // the previous tile's walk is done with the window and the rows
        const int32_t u_lo = a.g.u_lo[cur.side], u_hi = a.g.u_hi[cur.side];
        const int32_t c0 = u_lo * (u_lo - 1) / 2;
        const int32_t total = row_base(cur.dt, c0, u_lo, cur.b + 1);
#pragma unroll
        for (int i = 0; i < kRayMaxPer; ++i) {
            const int32_t g = (int32_t)threadIdx.x + i * kBlock;
            if (g < total) win[lds_pos(g)] = vals[i];
        }
        for (int32_t i = threadIdx.x; i <= cur.b - u_lo; i += kBlock) {
            const int32_t u = u_lo + i;
            RowRec rr;
            rr.kq = u_hi / u < a.s.H ? u_hi / u : a.s.H;   // harmonics inside the plane
            rr.kthr = (int32_t)((a.s.n_r - 1) / rr.kq);    // den > kthr <=> fewer than kq harmonics fit
            rr.T1 = row_base(cur.dt, c0, u_lo, u);
            rr.E = __umul24((uint32_t)cur.dt, (uint32_t)(u * u));
            rr.D1 = rr.E + __umul24((uint32_t)cur.dt, (uint32_t)(u * (u - 1) / 2)) + u;
            rr.rbase = u * cur.r0;
            rr.rowoff = ((int64_t)(cur.side ? -u : u) - a.s.z_min) * a.s.n_r;
            s_rows[i] = rr;
        }
        __syncthreads();
        const uint32_t tn = t + nw;
        Tile nxt = cur;
        if (tn < xe) {
            nxt = tile_at(a, tn, j);
            window_load<F16>(a, nxt, vals);
        }
        walk_tile<HMAX, GREEDY>(a, cur, win, s_tab, s_rows, valid, st);
        if (tn >= xe) break;
        t = tn;
        cur = nxt;
    }
    if (a.s.cand) stage_flush(st, a.s.cand, a.s.cap, a.s.count);
}

template <int HMAX>
const void *ray_kernel_h(bool greedy, bool f16) {
    if (greedy) return f16 ? (const void *)k_sum_2d_ray<HMAX, true, true> : (const void *)k_sum_2d_ray<HMAX, true, false>;
    return f16 ? (const void *)k_sum_2d_ray<HMAX, false, true> : (const void *)k_sum_2d_ray<HMAX, false, false>;
}

const void *ray_kernel(int hmax, bool greedy, bool f16) {
    switch (hmax) {
        case 4: return ray_kernel_h<4>(greedy, f16);
        case 8: return ray_kernel_h<8>(greedy, f16);
        case 16: return ray_kernel_h<16>(greedy, f16);
        case 32: return ray_kernel_h<32>(greedy, f16);
        default: return nullptr;
    }
}

}  // namespace

// Bands, then the tiles of both sides on a resident grid.  The caller
// checked ray_feasible and launches row z = 0 separately.
hipError_t launch_sum_2d_ray(Ray2dArgs a, int hmax, bool greedy, bool f16, int n_cu, hipStream_t st) {
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
    const void *fn = ray_kernel(hmax, greedy, f16);
    if (!fn) return hipErrorInvalidValue;
    const size_t lds = ray_window_bytes(a.g.budget, false) +
                       (a.s.cand ? sizeof(hs_candidate) * (kBlock / 64) * kRayStage : 0);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    uint32_t blocks = (uint32_t)per_cu * (uint32_t)(n_cu > 0 ? n_cu : 1);
    blocks -= blocks % (uint32_t)a.n_xcd;
    if (blocks < (uint32_t)a.n_xcd) blocks = (uint32_t)a.n_xcd;
    hipLaunchKernelGGL(k_ray_bands, dim3(1), dim3(kRayMaxBands), 0, st, a.g, a.bands);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&a};
    return hipLaunchKernel(fn, dim3(blocks), dim3(kBlock), args, lds, st);
}

}  // namespace hs
