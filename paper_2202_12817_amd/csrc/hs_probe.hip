// Gather-ceiling probe (measurement aid, libhs_probe.so): the greedy walk's
// access pattern -- per lane one fundamental n, per harmonic k the pair at
// k n + d with the drift update -- over a power-of-two working set, with no
// normalisation, SNR or output per fundamental.  Timing it on a set that stays
// in L2 and on one that does not gives the two line-traffic ceilings the
// harmonic-sum kernels are compared with.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hs_probe.h"

namespace {

constexpr int kK = 32;

typedef float f32x2_t __attribute__((ext_vector_type(2)));

// SET only names the regime in profiler output (0: a set of at most 8 MB,
// which every XCD's L2 holds; 1: at most 256 MB; 2: larger); the code is the
// same for all three.
template <int SET>
__global__ __launch_bounds__(256) void k_probe_gather(const float *x, uint32_t mask, int64_t n_fund, float *out) {
    // one buffer resource over the set plus the element after it (the pair
    // at position mask reads mask + 1)
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(x), (short)0, (int)((mask + 2u) * 4u), 0x00020000);
    const int64_t stride = (int64_t)gridDim.x * 256;
    float acc = 0.0f;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < n_fund; n += stride) {
        uint32_t m = (uint32_t)n, d = 0;
        float s = 0.0f;
#pragma unroll
        for (int k = 1; k <= kK; ++k) {
            const uint32_t p = (m + d) & mask;
            const f32x2_t w = __builtin_bit_cast(f32x2_t, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(p * 4u), 0, 0));
            const bool up = w.y > w.x;
            s += up ? w.y : w.x;
            d += up ? 1u : 0u;
            m += (uint32_t)n;
        }
        acc += s;
    }
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

}  // namespace

extern "C" int hsp_gather(const float *x, uint32_t mask, int64_t n_fund, int32_t blocks, float *out, void *stream) {
    if (!x || !out || blocks < 1 || n_fund < 1 || n_fund >= (1ll << 31) || mask == 0 || mask >= (1u << 28) ||
        (mask & (mask + 1u)) != 0)
        return (int)hipErrorInvalidValue;
    const uint32_t set = mask + 1u;
    auto kern = set <= (1u << 21) ? k_probe_gather<0> : set <= (1u << 26) ? k_probe_gather<1> : k_probe_gather<2>;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, x, mask, n_fund, out);
    return (int)hipGetLastError();
}
