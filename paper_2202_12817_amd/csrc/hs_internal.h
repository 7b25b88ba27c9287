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
    const double *user_norm;  // NULL or [2 groups] (mu1, sigma1)
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
};

// Harmonic sum over an f-fdot plane.
struct Sum2dArgs {
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

// Persistent XCD-aware batched harmonic sum (see hs_sum_xcd.hip).
struct XcdArgs {
    SumArgs s;                // offsets == NULL: one spectrum of s.n_bins
    int32_t n_spectra;
    int32_t n_xcd;            // virtual XCDs (work queues), >= 1
    uint32_t *tickets;        // [n_xcd] chunk counters, zero at launch
    uint32_t *prefix;         // [n_spectra + 1] chunk prefix, written by the launch
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
hipError_t launch_sum_2d(const Sum2dArgs &a, int hmax, bool greedy, bool f16, hipStream_t st);

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
    int last_groups;             // groups written by the most recent call
    uint32_t *tickets;           // device [kMaxXcd] work-queue counters of the persistent kernel
    uint32_t *prefix;            // device [max_groups + 1] chunk prefix of the persistent kernel
    int n_cu, n_xcd;             // device shape
    int xcd_f;                   // fundamentals per lane of the batched kernel
    int xcd_blocks;              // persistent grid of the batched kernel
    bool timing;                 // record stage events on every call
    std::vector<hipEvent_t> ev;  // 3 events per timed call: start, after norm, after sum
    int ev_used;                 // events of timed calls not yet read
};
