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

template <int HMAX, bool GREEDY, bool F16>
__global__ __launch_bounds__(kBlock) void k_sum_2d_ray(Ray2dArgs a) {
    using L = Loader<F16>;
    constexpr uint32_t eb = L::kBytes;
    extern __shared__ float win[];
    __shared__ int64_t s_r0, s_r1;
    __shared__ int32_t s_side, s_b;

    const uint32_t t = (blockIdx.x % (uint32_t)a.n_xcd) * a.per_xcd + blockIdx.x / (uint32_t)a.n_xcd;
    if (t >= a.n_tiles) return;   // uniform over the block
    if (threadIdx.x == 0) {
        int lo = 0, hi = a.n_bands - 1;   // last band with first_tile <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.bands[mid].first_tile <= t) lo = mid;
            else hi = mid - 1;
        }
        const RayBand bd = a.bands[lo];
        const int64_t r0 = bd.start + (int64_t)(t - bd.first_tile) * bd.delta;
        s_r0 = r0;
        s_r1 = r0 + bd.delta < bd.end ? r0 + bd.delta : bd.end;
        s_side = bd.side;
        s_b = bd.b;
    }
    __syncthreads();
    const int64_t r0 = uni64(s_r0);
    const int32_t dt = uni((int32_t)(s_r1 - r0));
    const int32_t side = uni(s_side), b = uni(s_b);
    const int32_t u_lo = a.g.u_lo[side], u_hi = a.g.u_hi[side];
    const int32_t sgn = side ? -1 : 1;
    const int64_t n_r = a.s.n_r;
    const int32_t c0 = (int32_t)tri(u_lo - 1);

    // 1. window rows u_lo..b, one wave per row at a time
    {
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int32_t m = u_lo + w; m <= b; m += kBlock / 64) {
            const int64_t col0 = (int64_t)m * r0;
            if (col0 > n_r - 1) continue;
            int64_t col1 = (int64_t)m * (r0 + dt);
            if (col1 > n_r - 1) col1 = n_r - 1;
            const int32_t len = (int32_t)(col1 - col0 + 1);
            const int64_t row = (int64_t)sgn * m - a.s.z_min;
            const __amdgpu_buffer_rsrc_t rs =
                make_rsrc((const char *)a.s.plane + row * a.s.stride * eb, (uint32_t)(n_r * eb));
            const int32_t base = dt * ((int32_t)tri(m - 1) - c0) + (m - u_lo);
            for (int32_t c = lane; c < len; c += 64) win[lds_pos(base + c)] = L::one(rs, (uint32_t)(col0 + c));
        }
    }
    __syncthreads();

    // 2. fundamentals of rows u_lo..b, consecutive lanes on consecutive columns
    const NormRec *nr = a.s.norm;
    const int valid = nr->valid;
    const float2 *tab = nr->t;
    const int64_t n_end = a.s.n_end < n_r ? a.s.n_end : n_r;
    const int32_t nf = dt * ((int32_t)tri(b) - c0);
    for (int32_t f0 = 0; f0 < nf; f0 += kBlock) {
        const int32_t f = f0 + (int32_t)threadIdx.x;
        int32_t u = u_lo, R = 0;
        if (f < nf) {
            const int32_t y = f / dt + c0;   // row u: the smallest with tri(u) > y
            u = (int32_t)((__builtin_sqrtf(8.0f * (float)y + 1.0f) - 1.0f) * 0.5f) + 1;
            while (tri(u) <= y) ++u;
            while (tri(u - 1) > y) --u;
            R = f - dt * ((int32_t)tri(u - 1) - c0);
        }
        const int64_t r = (int64_t)u * r0 + R;
        const bool in = f < nf && r < n_r;
        int K = 0;
        if (in && valid && r >= a.s.first_bin && r < n_end) {
            const uint32_t kk = (uint32_t)(n_r - 1) / (uint32_t)(GREEDY ? r + 1 : r);   // n_r < 2^30
            const int kz = u_hi / u;
            K = (int)kk < kz ? (int)kk : kz;
            if (K > a.s.H) K = a.s.H;
        }
        float S = 0.0f, best = 0.0f;
        int kb = 0, db = 0;
        int32_t d = 0;
#pragma unroll
        for (int k = 1; k <= HMAX; ++k) {
            if (k > K) break;
            const int32_t m = k * u;
            const int32_t g = dt * ((int32_t)tri(m - 1) - c0) + (m - u_lo) + k * R + d;
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
                if (kb == 0 || snr > best) {
                    best = snr;
                    kb = k;
                    db = d;
                }
            }
        }
        const Best bs{kb ? best : 0.0f, kb, db};
        const int64_t o = ((int64_t)sgn * u - a.s.z_min) * n_r + r;
        if (in) {
            if (a.s.snr) a.s.snr[o] = bs.snr;
            if (a.s.harm) a.s.harm[o] = (uint8_t)bs.harm;
            if (a.s.drift) a.s.drift[o] = (uint8_t)bs.drift;
        }
        if (a.s.cand)
            emit_candidate(in && bs.harm > 0 && bs.snr > a.s.thr, 0u, (uint32_t)o, bs, a.s.cand, a.s.cap, a.s.count);
    }
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
    const size_t lds = sizeof(float) * ((size_t)a.g.budget + ((size_t)a.g.budget >> 5) + 1);
    switch (hmax) {
        case 4: return ray_h<4>(a, greedy, f16, grid, lds, st);
        case 8: return ray_h<8>(a, greedy, f16, grid, lds, st);
        case 16: return ray_h<16>(a, greedy, f16, grid, lds, st);
        case 32: return ray_h<32>(a, greedy, f16, grid, lds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hs
