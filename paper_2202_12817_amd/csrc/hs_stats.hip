// Normalisation statistics of the harmonic sum (Sec. 2, Eq. (2): every
// partial sum is normalised by the mean and standard deviation of a sum of
// that many elements; the paper's GetMeanStdev, shared by all algorithms).
//
// Per group (a spectrum, or a whole f-fdot plane) the population mean and
// variance of the stored powers of bins [first_bin, N) are needed as the
// exact values rounded once to double.  k_stats streams each chunk once with
// 16-byte loads and accumulates sum x and sum x^2 in double-double (exact for
// powers whose magnitudes span fewer than ~50 binades, i.e. in practice);
// k_finalize reduces the chunk partials in a fixed order, rounds mean and
// variance once, takes a correctly rounded square root and writes the float
// tables rs_k = fl32(1/sigma_k), nm_k = fl32(-(mu_k/sigma_k)) for k = 1..32.
// Both kernels are FP64 (the only FP64 work of the path).
#include "hs_internal.h"

namespace hs {
namespace {

struct Group {
    const char *base;   // element 0 of the group
    int64_t rows, row_len, stride;
};

template <bool F16>
__device__ __forceinline__ Group group_of(const StatsArgs &a, int g) {
    constexpr int64_t eb = F16 ? 2 : 4;
    Group G;
    if (a.offsets) {
        int64_t off = a.offsets[g];
        G.base = (const char *)a.x + off * eb;
        G.rows = 1;
        G.row_len = a.offsets[g + 1] - off;
        if (G.row_len < 0 || G.row_len >= (1ll << 30)) G.row_len = 0;   // malformed offsets: nothing read
        G.stride = G.row_len;
    } else {
        G.base = (const char *)a.x;
        G.rows = a.rows;
        G.row_len = a.rows > 1 ? a.row_len : a.n_bins;
        G.stride = a.rows > 1 ? a.stride : a.n_bins;
    }
    return G;
}

template <bool F16>
__device__ __forceinline__ float elem_at(const char *x, int64_t e) {
    if constexpr (F16) {
        return (float)__builtin_bit_cast(_Float16, ((const unsigned short *)x)[e]);
    } else {
        return ((const float *)x)[e];
    }
}

__device__ __forceinline__ void acc1(dd &s1, dd &s2, float v) {
    double dv = (double)v;
    s1 = dd_add_d(s1, dv);
    s2 = dd_add_d(s2, dv * dv);      // the square of a float is exact in double
}

// Running sum x of 16-bit storage: every finite binary16 value is an integer
// multiple of 2^-24 of magnitude at most 2^40 - 2^29 in those units, so any
// sum of fewer than 8192 of them is an integer below 2^53 units and a plain
// double holds it exactly.  The partial sum is folded into the double-double
// sum every kFlush16 elements (one exact addition instead of a double-double
// step per element); sum x^2 keeps the double-double step.
constexpr int kFlush16 = 4096;

struct Part16 {
    double a1 = 0.0;   // exact partial sum x
    int cnt = 0;       // elements in a1
};

__device__ __forceinline__ void acc16(Part16 &p, dd &s2, float v) {
    const double dv = (double)v;
    p.a1 += dv;                      // exact (see above)
    s2 = dd_add_d(s2, dv * dv);      // the square of a float is exact in double
    ++p.cnt;
}

// Fold the partial sum once it holds kFlush16 elements or more (at most
// kFlush16 + 7: still far below the 8192 that keep it exact).
__device__ __forceinline__ void flush16(Part16 &p, dd &s1, int at_least) {
    if (p.cnt >= at_least) {
        s1 = dd_add_d(s1, p.a1);
        p.a1 = 0.0;
        p.cnt = 0;
    }
}

// Accumulate elements [lo, hi) of the array x (element units; x 16-byte
// aligned).  The full 16-byte vectors inside the range are read with vector
// loads, the ragged head and tail element by element, so nothing outside
// [lo, hi) is read.
template <bool F16>
__device__ __forceinline__ void accumulate(const char *x, int64_t lo, int64_t hi, dd &s1, dd &s2) {
    constexpr int64_t V = F16 ? 8 : 4;
    Part16 p;
    auto acc = [&](float v) {
        if constexpr (F16)
            acc16(p, s2, v);
        else
            acc1(s1, s2, v);
    };
    int64_t q0 = (lo + V - 1) / V, q1 = hi / V;
    if (q0 >= q1) {                          // no full vector: all element-wise
        for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) acc(elem_at<F16>(x, e));
    } else {
        for (int64_t e = lo + threadIdx.x; e < q0 * V; e += blockDim.x) acc(elem_at<F16>(x, e));
        for (int64_t e = q1 * V + threadIdx.x; e < hi; e += blockDim.x) acc(elem_at<F16>(x, e));
        const uint4 *vp = (const uint4 *)x;
        for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
            uint4 raw = vp[q];
            uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
            for (int j = 0; j < (int)V; ++j) {
                float v;
                if constexpr (F16) {
                    unsigned short b = (unsigned short)(w[j >> 1] >> ((j & 1) * 16));
                    v = (float)__builtin_bit_cast(_Float16, b);
                } else {
                    v = __builtin_bit_cast(float, w[j]);
                }
                acc(v);
            }
            if constexpr (F16) flush16(p, s1, kFlush16);
        }
    }
    if constexpr (F16) flush16(p, s1, 1);
}

template <bool F16>
__global__ __launch_bounds__(kBlock) void k_stats(StatsArgs a) {
    const int g = blockIdx.y, c = blockIdx.x;
    Group G = group_of<F16>(a, g);
    const int64_t f0 = a.first_bin;
    const int64_t W = G.row_len > f0 ? G.row_len - f0 : 0;   // counted bins per row
    const int64_t V = W * G.rows;                               // counted bins per group
    const int64_t v_lo = V * c / a.chunks, v_hi = V * (c + 1) / a.chunks;
    // element offsets are taken from the 16-byte aligned address at or below
    // the array start, so vector loads are aligned whatever x's alignment
    constexpr int64_t eb = F16 ? 2 : 4;
    const int64_t mis = (int64_t)(((uintptr_t)a.x & 15u) / eb);
    const char *xa = (const char *)a.x - mis * eb;
    const int64_t gofs = (G.base - (const char *)a.x) / eb + mis;
    dd s1{0.0, 0.0}, s2{0.0, 0.0};
    int64_t v = v_lo;
    while (v < v_hi) {                       // walk the rows the chunk covers
        int64_t r = v / W, col = f0 + v % W;
        int64_t n = W - (col - f0);
        if (n > v_hi - v) n = v_hi - v;
        int64_t e0 = gofs + r * G.stride + col;
        accumulate<F16>(xa, e0, e0 + n, s1, s2);
        v += n;
    }
    __shared__ dd sh1[kBlock], sh2[kBlock];
    sh1[threadIdx.x] = s1;
    sh2[threadIdx.x] = s2;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh1[threadIdx.x] = dd_add(sh1[threadIdx.x], sh1[threadIdx.x + s]);
            sh2[threadIdx.x] = dd_add(sh2[threadIdx.x], sh2[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        StatPart p{sh1[0].hi, sh1[0].lo, sh2[0].hi, sh2[0].lo};
        a.parts[(int64_t)g * a.chunks + c] = p;
    }
}

// One 64-lane block per group: fixed-order reduction of the chunk partials,
// mean / variance / sigma, then the float tables (lane k-1 writes entry k).
__global__ __launch_bounds__(64) void k_finalize(StatsArgs a) {
    const int g = blockIdx.x;
    const int lane = threadIdx.x;
    __shared__ dd sh1[64], sh2[64];
    __shared__ double s_mu, s_sigma;
    __shared__ int s_valid;
    if (a.user_norm == nullptr) {
        dd s1{0.0, 0.0}, s2{0.0, 0.0};
        for (int c = lane; c < a.chunks; c += 64) {
            StatPart p = a.parts[(int64_t)g * a.chunks + c];
            s1 = dd_add(s1, dd{p.s1hi, p.s1lo});
            s2 = dd_add(s2, dd{p.s2hi, p.s2lo});
        }
        sh1[lane] = s1;
        sh2[lane] = s2;
        __syncthreads();
        for (int s = 32; s > 0; s >>= 1) {
            if (lane < s) {
                sh1[lane] = dd_add(sh1[lane], sh1[lane + s]);
                sh2[lane] = dd_add(sh2[lane], sh2[lane + s]);
            }
            __syncthreads();
        }
        if (lane == 0) {
            int64_t rows = 1, row_len;
            if (a.offsets) {
                row_len = a.offsets[g + 1] - a.offsets[g];
                if (row_len < 0 || row_len >= (1ll << 30)) row_len = 0;
            } else {
                rows = a.rows;
                row_len = a.rows > 1 ? a.row_len : a.n_bins;
            }
            int64_t W = row_len > a.first_bin ? row_len - a.first_bin : 0;
            double M = (double)(W * rows);      // exact: counts < 2^53
            double mu = 0.0, sigma = 0.0;
            int valid = 0;
            if (W * rows > 0) {
                dd S1 = sh1[0], S2 = sh2[0];
                mu = dd_div_d(S1, M).hi;
                dd sq = dd_div_d(dd_mul(S1, S1), M);              // (sum x)^2 / M
                dd var = dd_div_d(dd_add(S2, dd_neg(sq)), M);     // population variance
                double v = var.hi;
                sigma = sqrt_rn(v);
                valid = (__builtin_isfinite(mu) && __builtin_isfinite(sigma) && sigma > 0.0) ? 1 : 0;
            }
            s_mu = mu;
            s_sigma = sigma;
            s_valid = valid;
        }
    } else if (a.user_table_h == 0) {
        if (lane == 0) {
            double mu = a.user_norm[2 * g], sigma = a.user_norm[2 * g + 1];
            s_mu = mu;
            s_sigma = sigma;
            s_valid = (__builtin_isfinite(mu) && __builtin_isfinite(sigma) && sigma > 0.0) ? 1 : 0;
        }
    } else {
        // the caller's per-k table [2][Ht] of this group: mu_1..mu_Ht, sigma_1..sigma_Ht;
        // usable only if every entry is finite and every sigma_k positive (one 64-lane wave)
        const int Ht = a.user_table_h;
        const double *row = a.user_norm + (int64_t)g * 2 * Ht;
        bool ok = true;
        if (lane < Ht) {
            const double m = row[lane], sg = row[Ht + lane];
            ok = __builtin_isfinite(m) && __builtin_isfinite(sg) && sg > 0.0;
        }
        const bool all_ok = __ballot(!ok) == 0ull;
        if (lane == 0) {
            s_mu = row[0];
            s_sigma = row[Ht];
            s_valid = all_ok ? 1 : 0;
        }
    }
    __syncthreads();
    NormRec *rec = a.norm + g;
    const double mu1 = s_mu, sigma1 = s_sigma;
    const int valid = s_valid;
    if (lane == 0) {
        rec->mu1 = mu1;
        rec->sigma1 = sigma1;
        rec->valid = valid;
    }
    if (lane < HS_MAX_HARMONICS) {
        float rs = 0.0f, nm = 0.0f;
        if (valid && a.user_table_h > 0) {
            if (lane < a.user_table_h) {
                const double *row = a.user_norm + (int64_t)g * 2 * a.user_table_h;
                const double mu_k = row[lane], sig_k = row[a.user_table_h + lane];
                rs = (float)(1.0 / sig_k);
                nm = (float)(-(mu_k / sig_k));
            }
        } else if (valid) {
            const double k = (double)(lane + 1);
            const double mu_k = k * mu1;
            const double sig_k = sqrt_rn(k) * sigma1;
            rs = (float)(1.0 / sig_k);
            nm = (float)(-(mu_k / sig_k));
        }
        rec->t[lane] = make_float2(rs, nm);
        if (a.tab_t) a.tab_t[(int64_t)lane * a.tab_stride + g] = make_float2(rs, nm);
    }
}

__global__ void k_export_norm(const NormRec *norm, int n, int H, double *mu_sigma, float *tables,
                              int32_t *valid) {
    const int g = blockIdx.x;
    const int lane = threadIdx.x;
    if (g >= n) return;
    const NormRec *r = norm + g;
    if (lane == 0) {
        if (mu_sigma) {
            mu_sigma[2 * g] = r->mu1;
            mu_sigma[2 * g + 1] = r->sigma1;
        }
        if (valid) valid[g] = r->valid;
    }
    if (tables && lane < H) {
        tables[(int64_t)g * 2 * H + lane] = r->t[lane].x;
        tables[(int64_t)g * 2 * H + H + lane] = r->t[lane].y;
    }
}

__global__ void k_zero_u64(unsigned long long *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

__global__ void k_zero_u32(uint32_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_quantize_f16(const float *x, int64_t n, float scale, uint16_t *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float y = x[i] / scale;                        // correctly rounded float division
        y = y > 65504.0f ? 65504.0f : (y < -65504.0f ? -65504.0f : y);
        _Float16 h = (_Float16)y;                      // round to nearest even
        out[i] = __builtin_bit_cast(uint16_t, h);
    }
}

}  // namespace

hipError_t launch_stats(const StatsArgs &a, int groups, bool f16, hipStream_t st) {
    dim3 grid(a.chunks, groups);
    if (f16)
        hipLaunchKernelGGL(k_stats<true>, grid, dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL(k_stats<false>, grid, dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_finalize(const StatsArgs &a, int groups, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(groups), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_export_norm(const NormRec *norm, int n, int H, double *mu_sigma, float *tables,
                              int32_t *valid, hipStream_t st) {
    hipLaunchKernelGGL(k_export_norm, dim3(n), dim3(64), 0, st, norm, n, H, mu_sigma, tables, valid);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_quantize_f16(const float *x, int64_t n, float scale, uint16_t *out, hipStream_t st) {
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_quantize_f16, dim3((unsigned)blocks), dim3(kBlock), 0, st, x, n, scale, out);
    return hipGetLastError();
}

}  // namespace hs
