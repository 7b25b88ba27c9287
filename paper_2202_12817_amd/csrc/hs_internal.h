// Host-side declarations shared by the harmonic-sum library's translation
// units: the plan, the kernel argument blocks and the launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hs.h"
#include "hs_device.h"

namespace hs {

constexpr int kBlock = 256;          // threads per harmonic-sum / statistics block
constexpr int kChunksBatched = 64;   // statistics chunks per spectrum of a batch
constexpr int kChunks1D = 512;       // statistics chunks of a single spectrum
constexpr int kChunks2D = 2048;      // statistics chunks of a plane
constexpr int kTileBlocksBatched = 96;   // plain kernel: blocks per spectrum of a batch
constexpr int64_t kPlainBlocks = 32768;  // plain kernel: most workgroups of a 1D or plane launch (tiles loop
                                         // within; 16k..128k measured alike on the plane workload)
constexpr int kMaxXcd = 64;              // work-queue counters in the plan workspace

// Where the statistics of group g (spectrum or plane) come from: `rows` rows
// of `row_len` powers, row r starting at element base(g) + r * stride, bins
// [first_bin, row_len) of every row counted.
struct StatsArgs {
    const void *x;
    const int64_t *offsets;   // batched: group g = spectrum g; else NULL
    int64_t n_bins;           // 1D length (offsets == NULL, rows == 1)
    int64_t rows;             // 2D: rows per plane (1 otherwise)
    int64_t row_len;          // 2D: columns
    int64_t stride;           // 2D: row stride in elements
    int32_t first_bin;
    int32_t chunks;           // chunks per group
    StatPart *parts;          // [groups][chunks]
    NormRec *norm;            // [groups]
    const double *user_norm;  // NULL, or [groups][2] (mu1, sigma1), or [groups][2][user_table_h] (mu_k, sigma_k)
    int32_t user_table_h;     // 0: user_norm holds (mu1, sigma1) pairs; H: per-k tables of H entries
    int32_t il_spectra;       // interleaved layout: spectra per row (group g = spectrum g of n_bins bins)
    float2 *tab_t;            // NULL, or also write (rs_k, nm_k) of group g to tab_t[(k-1) tab_stride + g]
    int32_t tab_stride;
};

// Harmonic sum over 1D spectra (one, or a batch through `offsets`).
struct SumArgs {
    const void *x;
    const int64_t *offsets;   // NULL: one spectrum of n_bins
    int64_t n_bins;
    const NormRec *norm;
    int32_t first_bin;
    int32_t H;
    int64_t n_end;            // fundamentals >= n_end give zeros (already >= 1)
    uint64_t kmask;           // eligible partial sums (bit k-1)
    uint64_t report_mask;     // partial sums to export (1D only)
    float *partial;
    float *snr;
    uint8_t *harm;
    uint8_t *drift;
    hs_candidate *cand;
    int64_t cap;
    unsigned long long *count;
    float thr;
    int32_t n_xcd;            // batched plain launches: XCDs the workgroups are dealt to (1: no remap)
};

// Workgroup (blockIdx.x, blockIdx.y) of a (gridDim.x, gridDim.y) grid as
// (tile block, spectrum) of a batched plain launch.  The dispatcher deals
// workgroups to the XCDs in turn by linear id, so workgroup L runs on XCD
// L mod n_xcd; renumbering L to (L mod n_xcd) (T / n_xcd) + L / n_xcd gives
// each XCD a contiguous run of whole spectra, which it walks in order, so
// one XCD's L2 holds the harmonic windows of a few spectra instead of every
// XCD holding a slice of every spectrum.  A bijection: results do not change.
__device__ __forceinline__ void batched_block(int n_xcd, int *bx, int *spectrum) {
    const uint32_t gx = gridDim.x, T = gridDim.x * gridDim.y;
    uint32_t L = blockIdx.x + blockIdx.y * gx;
    if (n_xcd > 1 && T % (uint32_t)n_xcd == 0) L = (L % (uint32_t)n_xcd) * (T / (uint32_t)n_xcd) + L / (uint32_t)n_xcd;
    *bx = (int)(L % gx);
    *spectrum = (int)(L / gx);
}

// Harmonic sum over an f-fdot plane.
struct Sum2dArgs {
    int32_t row0;             // plain kernel: first plane row of the launch (blockIdx.y = row - row0)
    const void *plane;
    int64_t n_r;
    int64_t stride;
    int32_t z_min, z_max;
    const NormRec *norm;
    int32_t first_bin;
    int32_t H;
    int64_t n_end;
    uint64_t kmask;
    float *snr;
    uint8_t *harm;
    uint8_t *drift;
    hs_candidate *cand;
    int64_t cap;
    unsigned long long *count;
    float thr;
};

// Harmonic sum over equal-length spectra in the interleaved layout
// x[m n_spectra + s] (see hs_interleaved.hip).
struct IlArgs {
    const void *x;
    int64_t n_bins;
    int32_t n_spectra;
    const NormRec *norm;      // [n_spectra]
    const float2 *tab_t;      // (rs_k, nm_k) of spectrum s at tab_t[(k-1) tab_stride + s]
    int32_t tab_stride;
    int32_t first_bin;
    int32_t H;
    int64_t n_end;
    uint64_t kmask;
    float *snr;               // NULL or [n_bins][n_spectra]
    uint8_t *harm;
    uint8_t *drift;
    hs_candidate *cand;
    int64_t cap;
    unsigned long long *count;
    float thr;
    int32_t n_groups;         // spectra groups of 64 lanes
    int32_t tile;             // fundamentals per wave task
    int64_t n_tasks;          // n_groups * tiles
    int32_t n_xcd;
};

// Peak clustering of dense outputs (see hs_pipeline.hip).
struct PeakArgs {
    const float *snr;
    const uint8_t *harm;
    const uint8_t *drift;     // NULL: drift 0 in the records
    const int64_t *offsets;   // NULL: one spectrum of n_bins
    int64_t n_bins;
    int64_t radius;
    float thr;
    hs_candidate *cand;
    int64_t cap;
    unsigned long long *count;
};

// Persistent XCD-aware batched harmonic sum (see hs_sum_xcd.hip).
struct XcdArgs {
    SumArgs s;                // offsets == NULL: one spectrum of s.n_bins
    int32_t n_spectra;
    int32_t n_xcd;            // virtual XCDs (work queues), >= 1
    uint32_t *tickets;        // [n_xcd] chunk counters, zero at launch
    uint32_t *prefix;         // [n_spectra + 1] chunk prefix, written by the launch
};

// Ray-tiled f-fdot plane (see hs_sum_2d_ray.hip).  Rows z != 0 form two
// sides (z > 0 and z < 0) of rows u = |z| in [u_lo, u_hi]; a tile of a side
// is a ratio range [r0, r0 + delta) and holds the fundamentals (u, r) with
// u r0 <= r < u (r0 + delta); its harmonics read row m = k u only at columns
// [m r0, m (r0 + delta)], so the tile's window of rows u_lo..b is staged once.
constexpr int kRayLdsBytes = 22 * 1024;   // LDS of one tile's staged window (default; 5 workgroups per CU)
constexpr int kRayMaxPer = 24;            // window elements per thread: budget <= 256 kRayMaxPer
constexpr int kRayMaxBands = 512;    // bands of both sides (a band: tiles with the same top row b)
constexpr int kRayMaxRows = 160;     // rows |z| of one side

struct RayGeom {
    int64_t n_r;
    int32_t u_lo[2], u_hi[2];   // side 0: z = +u, side 1: z = -u; u_lo > u_hi: empty side
    int32_t budget;             // window elements (floats) per tile, <= 256 kRayMaxPer
};

struct RayBand {
    uint32_t first_tile;        // tiles of the band: [first_tile, first_tile + tiles)
    int32_t side;
    int32_t b;                  // highest window row of the band's tiles
    int32_t delta;              // tile width (ratio units)
    int64_t start, end;         // ratio range of the band
};

__host__ __device__ inline int64_t tri(int64_t x) { return x * (x + 1) / 2; }

// Staged window: budget elements (floats, or float pairs), one pad element
// per 32, rounded to 16 bytes.
__host__ __device__ inline size_t ray_window_bytes(int budget, bool greedy) {
    const size_t n = (size_t)budget + ((size_t)budget >> 5) + 1;
    return (n * (greedy ? 8 : 4) + 15) & ~(size_t)15;
}

// Largest budget whose window fits lds_bytes.
inline int ray_budget_for(int lds_bytes, bool greedy) {
    int e = lds_bytes / (greedy ? 8 : 4);
    while (e > 0 && ray_window_bytes(e, greedy) > (size_t)lds_bytes) --e;
    return e;
}

__host__ __device__ inline int ray_side_bands(const RayGeom &g, int side) {
    return g.u_lo[side] <= g.u_hi[side] ? g.u_hi[side] - g.u_lo[side] + 1 : 0;
}

// Band j of a side (top row b = u_hi - j): ratio range and tile width; returns
// the number of tiles (0 for an empty band).  Band b covers the ratios whose
// highest non-empty window row is b: ratios r0 with floor((n_r - 1) / r0) = b
// (for b = u_hi: every r0 <= (n_r - 1) / u_hi, including 0).
__host__ __device__ inline uint32_t ray_band(const RayGeom &g, int side, int j, int64_t *start, int64_t *end,
                                             int32_t *delta) {
    const int64_t lo = g.u_lo[side], hi = g.u_hi[side], b = hi - j;
    const int64_t rho_end = (g.n_r + lo - 1) / lo;   // every column r < n_r of every row u >= lo
    const int64_t s = b == hi ? 0 : (g.n_r - 1) / (b + 1) + 1;
    int64_t e = (g.n_r - 1) / b + 1;
    if (e > rho_end) e = rho_end;
    const int64_t rows = b - lo + 1, t = tri(b) - tri(lo - 1);
    int64_t d = (g.budget - rows) / t;
    if (d < 1) d = 1;
    *start = s;
    *end = e;
    *delta = (int32_t)d;
    return s < e ? (uint32_t)((e - s + d - 1) / d) : 0u;
}

// Every tile's window fits the budget (a tile of width 1 of the widest band).
__host__ __device__ inline bool ray_feasible(const RayGeom &g) {
    for (int side = 0; side < 2; ++side) {
        if (g.u_lo[side] > g.u_hi[side]) continue;
        const int64_t lo = g.u_lo[side], hi = g.u_hi[side];
        if (tri(hi) - tri(lo - 1) + (hi - lo + 1) > g.budget) return false;
        if (hi - lo + 1 > kRayMaxRows) return false;
    }
    return ray_side_bands(g, 0) + ray_side_bands(g, 1) <= kRayMaxBands;
}

struct Ray2dArgs {
    Sum2dArgs s;
    RayGeom g;
    RayBand *bands;             // [n_bands], written by the band kernel of the same launch sequence
    int32_t n_bands;
    uint32_t n_tiles;
    int32_t n_xcd;              // XCD q owns tiles [n_tiles q / n_xcd, n_tiles (q + 1) / n_xcd)
};

hipError_t launch_stats(const StatsArgs &a, int groups, bool f16, hipStream_t st);
hipError_t launch_finalize(const StatsArgs &a, int groups, hipStream_t st);
hipError_t launch_export_norm(const NormRec *norm, int n, int H, double *mu_sigma, float *tables,
                              int32_t *valid, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long *p, hipStream_t st);
hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t st);
hipError_t xcd_resident_blocks(int hmax, bool greedy, bool f16, int F, int *per_cu);
hipError_t launch_sum_xcd(const XcdArgs &a, int hmax, bool greedy, bool f16, int F, int blocks, hipStream_t st);
hipError_t launch_quantize_f16(const float *x, int64_t n, float scale, uint16_t *out, hipStream_t st);
hipError_t launch_sum_1d(const SumArgs &a, int hmax, bool greedy, bool f16, dim3 grid, hipStream_t st);
hipError_t launch_sum_2d(const Sum2dArgs &a, int hmax, bool greedy, bool f16, int rows, hipStream_t st);
hipError_t launch_sum_2d_ray(Ray2dArgs a, int hmax, bool greedy, bool f16, int n_cu, hipStream_t st);
hipError_t launch_presto(const SumArgs &a, int hmax, int variant, bool f16, dim3 grid, hipStream_t st);
hipError_t launch_stats_il(const StatsArgs &a, bool f16, hipStream_t st);
hipError_t launch_sum_il(const IlArgs &a, int hmax, bool greedy, bool f16, hipStream_t st);
hipError_t launch_interleave(const void *x, int64_t n_bins, int n_spectra, int elem_bytes, void *out, hipStream_t st);
hipError_t launch_power(const void *fft, int64_t n, bool interbin, float sc, float sch, float *out, hipStream_t st);
hipError_t launch_peaks(const PeakArgs &a, int groups, int64_t max_len, hipStream_t st);

}  // namespace hs

#include <vector>

struct hs_plan {
    hs_plan_desc desc;
    int device;
    int hmax;                    // compiled harmonic bucket >= desc.harmonics
    int max_groups;              // norm records available
    int parts_cap;               // StatPart records available
    hs::NormRec *norm;           // device [max_groups]
    hs::StatPart *parts;         // device [parts_cap]
    char *ws;                    // device workspace (one block; the pointers below are carved from it)
    bool ws_owned;               // allocated by the plan (else the caller's)
    int last_groups;             // groups written by the most recent call
    uint32_t *tickets;           // device [kMaxXcd] work-queue counters of the persistent kernel
    uint32_t *prefix;            // device [max_groups + 1] chunk prefix of the persistent kernel
    hs::RayBand *ray;            // device [kRayMaxBands] band table of the ray-tiled plane kernel
    float2 *tab_t;               // device [HS_MAX_HARMONICS][max_groups] tables, spectrum fastest (interleaved walk)
    int n_cu, n_xcd;             // device shape
    int xcd_f;                   // fundamentals per lane of the batched kernel
    int xcd_blocks;              // persistent grid of the batched kernel
    bool batched_plain;          // AUTO plans: batches run the plain kernel (chosen by the tuner)
    int tile_blocks;             // batched plain launches: workgroups per spectrum
    int ray_lds;                 // LDS bytes of a tile's window in the ray-tiled plane kernel
    bool timing;                 // record stage events on every call
    std::vector<hipEvent_t> ev;  // 3 events per timed call: start, after norm, after sum
    int ev_used;                 // events of timed calls not yet read

    // Whole-call hipGraph replay: each distinct argument set of a sum call is
    // captured once (on cap_stream, which only records) and replayed on the
    // caller's stream afterwards.
    struct GraphEntry {
        std::vector<uint64_t> key;  // entry point and every argument of the call
        hipGraphExec_t exec;
        hipEvent_t done;            // recorded after the latest replay
        uint64_t last_use;
    };
    bool graph;
    hipStream_t cap_stream;
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock;
    int64_t captures, replays;
};
