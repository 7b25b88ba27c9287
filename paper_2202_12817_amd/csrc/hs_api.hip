// C ABI of the harmonic-sum library: argument validation, plan/workspace
// management and the launch sequence of every entry point (declared and
// documented in include/hs.h).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>

#include "hs_internal.h"

namespace {

// The calling thread's last failure message: a fixed buffer, so recording an
// error never allocates (and never throws).
thread_local char g_last_error[512];

hs_status fail(hs_status s, const char *msg) {
    snprintf(g_last_error, sizeof g_last_error, "%s", msg);
    return s;
}

hs_status fail_hip(hipError_t e, const char *where) {
    snprintf(g_last_error, sizeof g_last_error, "%s: %s", where, hipGetErrorString(e));
    return HS_ERR_HIP;
}

// Every entry point runs its body through this: no C++ exception crosses the
// C ABI (a failed host allocation inside the library, e.g. of the graph
// cache or the tuner's strings, becomes HS_ERR_NOMEM).
template <class Body>
hs_status guarded(Body &&body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(HS_ERR_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(HS_ERR_INTERNAL, "unexpected exception inside the library");
    }
}

int bucket(int H) {
    if (H <= 4) return 4;
    if (H <= 8) return 8;
    if (H <= 16) return 16;
    if (H <= 32) return 32;
    return 64;
}

// natural alignment of the stored powers
bool aligned_elem(const void *p, int dtype) { return ((uintptr_t)p & (dtype == HS_F16 ? 1u : 3u)) == 0; }

uint64_t eligible_mask(const hs_plan_desc &d) {
    const uint64_t all = d.harmonics >= 64 ? ~0ull : ((1ull << d.harmonics) - 1ull);
    return d.harmonic_mask ? (d.harmonic_mask & all) : all;
}

// The PRESTO-style comparators (last-bin indexing, one kernel).
bool is_presto(int mode) { return mode == HS_PRESTO || mode == HS_PRESTO_ALL || mode == HS_PRESTO_PLUS; }

int64_t n_end_of(const hs_plan_desc &d, int64_t len) {
    return d.fundamental_end > 0 && d.fundamental_end < len ? d.fundamental_end : len;
}

// Stage events of a timed call: index 0 before the normalisation stage, 1
// after it, 2 after the harmonic-sum kernel.
hs_status mark(hs_plan *p, int stage, hipStream_t st) {
    if (!p->timing) return HS_OK;
    if (stage == 0 && p->ev_used + 3 > (int)p->ev.size()) {
        for (int i = 0; i < 3; ++i) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return fail_hip(r, "hipEventCreate");
            p->ev.push_back(e);
        }
    }
    hipError_t r = hipEventRecord(p->ev[p->ev_used + stage], st);
    if (r != hipSuccess) return fail_hip(r, "hipEventRecord");
    if (stage == 2) p->ev_used += 3;
    return HS_OK;
}

// The persistent kernel over n spectra (offsets == NULL: one spectrum of
// a.n_bins).
hs_status run_persistent(hs_plan *p, const hs::SumArgs &a, int n, hipStream_t st) {
    hs::XcdArgs xa{};
    xa.s = a;
    xa.n_spectra = n;
    xa.n_xcd = p->n_xcd;
    xa.tickets = p->tickets;
    xa.prefix = p->prefix;
    hipError_t e = hs::launch_zero_u32(p->tickets, p->n_xcd, st);
    if (e != hipSuccess) return fail_hip(e, "ticket reset");
    e = hs::launch_sum_xcd(xa, p->hmax, p->desc.mode == HS_GREEDY, p->desc.dtype == HS_F16, p->xcd_f,
                           p->xcd_blocks, st);
    if (e != hipSuccess) return fail_hip(e, "harmonic-sum kernel");
    return HS_OK;
}

// Statistics and tables of `groups` groups (or the caller's normalisation).
hs_status run_norm(hs_plan *p, hs::StatsArgs sa, int groups, hipStream_t st) {
    hipError_t e;
    hs_status ms = mark(p, 0, st);
    if (ms != HS_OK) return ms;
    sa.parts = p->parts;
    sa.norm = p->norm;
    if (sa.user_norm == nullptr) {
        if ((int64_t)groups * sa.chunks > p->parts_cap) return fail(HS_ERR_ARG, "too many statistics chunks");
        e = sa.il_spectra ? hs::launch_stats_il(sa, p->desc.dtype == HS_F16, st)
                          : hs::launch_stats(sa, groups, p->desc.dtype == HS_F16, st);
        if (e != hipSuccess) return fail_hip(e, "statistics kernel");
    }
    e = hs::launch_finalize(sa, groups, st);
    if (e != hipSuccess) return fail_hip(e, "finalise kernel");
    p->last_groups = groups;
    return mark(p, 1, st);
}

int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

hs_status resident_limit(hs_plan *p, int F, int *per_cu);

// Shape of the persistent batched launch: one work queue per XCD, as many
// workgroups as are resident.  HS_XCD_F and HS_XCD_WGS_PER_CU override the
// defaults (tuning aids).
hs_status setup_xcd(hs_plan *p) {
    hipError_t e = hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) return fail_hip(e, "hipDeviceGetAttribute(CUs)");
    int nx = 0;
    if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, p->device) != hipSuccess || nx < 1) {
        (void)hipGetLastError();
        nx = 1;
    }
    if (nx > hs::kMaxXcd) nx = hs::kMaxXcd;
    p->n_xcd = nx;
    // default shape: what the tuner picks on the 512-spectrum batch (FP32:
    // 2 fundamentals per lane, 4 workgroups per CU; FP16: 4 and 5), capped
    // by the occupancy; hs_plan_tune_batched searches up to that limit
    const bool f16 = p->desc.dtype == HS_F16;
    const int F0 = f16 ? 4 : 2;
    int F = env_int("HS_XCD_F", F0);
    p->xcd_f = (F == 1 || F == 2 || F == 4) ? F : F0;
    int per_cu = 0;
    hs_status s = resident_limit(p, p->xcd_f, &per_cu);
    if (s != HS_OK) return s;
    int want = env_int("HS_XCD_WGS_PER_CU", f16 ? 5 : 4);
    if (want >= 1 && want < per_cu) per_cu = want;
    p->xcd_blocks = per_cu * p->n_cu;
    // LDS bytes of a tile's window in the ray-tiled plane kernel (HS_RAY_LDS
    // overrides: 4096..61440, so that window and staging stay below 64 KiB)
    const int rl = env_int("HS_RAY_LDS", hs::kRayLdsBytes);
    p->ray_lds = rl >= 4096 && rl <= 61440 ? rl : hs::kRayLdsBytes;
    // workgroups per spectrum of the batched plain launches (HS_TILE_BLOCKS
    // overrides: 8..4096)
    const int tb = env_int("HS_TILE_BLOCKS", hs::kTileBlocksBatched);
    p->tile_blocks = tb >= 8 && tb <= 4096 ? tb : hs::kTileBlocksBatched;
    return HS_OK;
}

// Launch sequences of the sum entry points (arguments already validated).
hs_status enqueue_1d(hs_plan *p, const void *x, int64_t n_bins, const double *norm, float *snr, uint8_t *harm,
                     uint8_t *drift, float *partial, hipStream_t st) {
    hs::StatsArgs sa{};
    sa.x = x;
    sa.offsets = nullptr;
    sa.n_bins = n_bins;
    sa.rows = 1;
    sa.row_len = n_bins;
    sa.stride = n_bins;
    sa.first_bin = p->desc.first_bin;
    sa.chunks = hs::kChunks1D;
    sa.user_norm = norm;
    sa.user_table_h = norm && p->desc.norm_kind == HS_NORM_TABLE ? p->desc.harmonics : 0;
    hs_status s = run_norm(p, sa, 1, st);
    if (s != HS_OK) return s;
    hs::SumArgs a{};
    a.x = x;
    a.offsets = nullptr;
    a.n_bins = n_bins;
    a.norm = p->norm;
    a.first_bin = p->desc.first_bin;
    a.H = p->desc.harmonics;
    a.n_end = n_end_of(p->desc, n_bins);
    a.kmask = eligible_mask(p->desc);
    a.report_mask = partial ? p->desc.report_mask : 0;
    a.partial = p->desc.report_mask ? partial : nullptr;
    a.snr = snr;
    a.harm = harm;
    a.drift = drift;
    a.cand = nullptr;
    a.thr = p->desc.threshold;
    // AUTO: the plain kernel, measured faster than the persistent one on a
    // single spectrum at every size from 2^14 to 2^28 bins
    const bool plain = p->desc.kernel != HS_KERNEL_PERSISTENT;
    if (is_presto(p->desc.mode)) {
        int64_t blocks = (n_bins + hs::kBlock - 1) / hs::kBlock;
        if (blocks > hs::kPlainBlocks) blocks = hs::kPlainBlocks;
        hipError_t e = hs::launch_presto(a, p->hmax, p->desc.mode, p->desc.dtype == HS_F16, dim3((unsigned)blocks, 1),
                                         st);
        if (e != hipSuccess) return fail_hip(e, "PRESTO-style sum kernel");
    } else if (plain || a.partial) {
        int64_t blocks = (n_bins + hs::kBlock - 1) / hs::kBlock;   // tiles loop within the grid
        if (blocks > hs::kPlainBlocks) blocks = hs::kPlainBlocks;
        dim3 grid((unsigned)blocks, 1);
        hipError_t e = hs::launch_sum_1d(a, p->hmax, p->desc.mode == HS_GREEDY, p->desc.dtype == HS_F16, grid, st);
        if (e != hipSuccess) return fail_hip(e, "harmonic-sum kernel");
    } else {
        s = run_persistent(p, a, 1, st);
        if (s != HS_OK) return s;
    }
    return mark(p, 2, st);
}

hs_status enqueue_batched(hs_plan *p, const void *x, const int64_t *offsets, int32_t n_spectra, const double *norm,
                          float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand, int64_t cand_capacity,
                          unsigned long long *cand_count, hipStream_t st) {
    hipError_t e;
    if (cand) {
        e = hs::launch_zero_u64(cand_count, st);
        if (e != hipSuccess) return fail_hip(e, "counter reset");
    }
    hs::StatsArgs sa{};
    sa.x = x;
    sa.offsets = offsets;
    sa.rows = 1;
    sa.first_bin = p->desc.first_bin;
    sa.chunks = hs::kChunksBatched;
    sa.user_norm = norm;
    sa.user_table_h = norm && p->desc.norm_kind == HS_NORM_TABLE ? p->desc.harmonics : 0;
    hs_status s = run_norm(p, sa, n_spectra, st);
    if (s != HS_OK) return s;
    hs::SumArgs a{};
    a.x = x;
    a.offsets = offsets;
    a.n_bins = 0;
    a.norm = p->norm;
    a.first_bin = p->desc.first_bin;
    a.H = p->desc.harmonics;
    a.n_end = p->desc.fundamental_end > 0 ? p->desc.fundamental_end : (1ll << 62);
    a.kmask = eligible_mask(p->desc);
    a.report_mask = 0;
    a.partial = nullptr;
    a.snr = snr;
    a.harm = harm;
    a.drift = drift;
    a.cand = cand;
    a.cap = cand_capacity;
    a.count = cand_count;
    a.thr = p->desc.threshold;
    a.n_xcd = p->n_xcd;
    if (is_presto(p->desc.mode)) {
        e = hs::launch_presto(a, p->hmax, p->desc.mode, p->desc.dtype == HS_F16,
                              dim3((unsigned)p->tile_blocks, (unsigned)n_spectra), st);
        if (e != hipSuccess) return fail_hip(e, "PRESTO-style sum kernel");
    } else if (p->desc.kernel == HS_KERNEL_PLAIN || (p->desc.kernel == HS_KERNEL_AUTO && p->batched_plain)) {
        dim3 grid((unsigned)p->tile_blocks, (unsigned)n_spectra);
        e = hs::launch_sum_1d(a, p->hmax, p->desc.mode == HS_GREEDY, p->desc.dtype == HS_F16, grid, st);
        if (e != hipSuccess) return fail_hip(e, "harmonic-sum kernel");
    } else {
        s = run_persistent(p, a, n_spectra, st);
        if (s != HS_OK) return s;
    }
    return mark(p, 2, st);
}

hs_status enqueue_2d(hs_plan *p, const void *plane, int64_t n_r, int64_t row_stride, int32_t z_min, int32_t z_max,
                     const double *norm, float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand,
                     int64_t cand_capacity, unsigned long long *cand_count, hipStream_t st) {
    const int64_t n_z = (int64_t)z_max - z_min + 1;
    hipError_t e;
    if (cand) {
        e = hs::launch_zero_u64(cand_count, st);
        if (e != hipSuccess) return fail_hip(e, "counter reset");
    }
    hs::StatsArgs sa{};
    sa.x = plane;
    sa.offsets = nullptr;
    sa.n_bins = n_r;
    sa.rows = n_z;
    sa.row_len = n_r;
    sa.stride = row_stride;
    sa.first_bin = p->desc.first_bin;
    sa.chunks = hs::kChunks2D;
    sa.user_norm = norm;
    sa.user_table_h = norm && p->desc.norm_kind == HS_NORM_TABLE ? p->desc.harmonics : 0;
    hs_status s = run_norm(p, sa, 1, st);
    if (s != HS_OK) return s;
    hs::Sum2dArgs a{};
    a.row0 = 0;
    a.plane = plane;
    a.n_r = n_r;
    a.stride = row_stride;
    a.z_min = z_min;
    a.z_max = z_max;
    a.norm = p->norm;
    a.first_bin = p->desc.first_bin;
    a.H = p->desc.harmonics;
    a.n_end = n_end_of(p->desc, n_r);
    a.kmask = eligible_mask(p->desc);
    a.snr = snr;
    a.harm = harm;
    a.drift = drift;
    a.cand = cand;
    a.cap = cand_capacity;
    a.count = cand_count;
    a.thr = p->desc.threshold;
    const bool greedy = p->desc.mode == HS_GREEDY, f16 = p->desc.dtype == HS_F16;
    hs::RayGeom g{};
    g.n_r = n_r;
    g.u_lo[0] = z_min > 1 ? z_min : 1;
    g.u_hi[0] = z_max;
    g.u_lo[1] = -z_max > 1 ? -z_max : 1;
    g.u_hi[1] = -z_min;
    g.budget = hs::ray_budget_for(p->ray_lds, false);
    if (g.budget > hs::kBlock * hs::kRayMaxPer) g.budget = hs::kBlock * hs::kRayMaxPer;
    if (p->desc.kernel == HS_KERNEL_PERSISTENT && p->hmax <= 32 && hs::ray_feasible(g)) {
        hs::Ray2dArgs ra{};
        ra.s = a;
        ra.g = g;
        ra.bands = p->ray;
        ra.n_xcd = p->n_xcd;
        e = hs::launch_sum_2d_ray(ra, p->hmax, greedy, f16, p->n_cu, st);
        if (e != hipSuccess) return fail_hip(e, "harmonic-sum kernel (ray tiles)");
        if (z_min <= 0 && z_max >= 0) {   // row z = 0
            a.row0 = -z_min;
            e = hs::launch_sum_2d(a, p->hmax, greedy, f16, 1, st);
        }
    } else {
        e = hs::launch_sum_2d(a, p->hmax, greedy, f16, (int)n_z, st);
    }
    if (e != hipSuccess) return fail_hip(e, "harmonic-sum kernel");
    return mark(p, 2, st);
}

// Equal-length spectra in the interleaved layout: statistics per spectrum
// (column), then one launch of the interleaved walk.
constexpr int kIlTile = 32;   // fundamentals per wave task of the interleaved walk

hs_status enqueue_interleaved(hs_plan *p, const void *x, int64_t n_bins, int32_t n_spectra, const double *norm,
                              float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand, int64_t cand_capacity,
                              unsigned long long *cand_count, hipStream_t st) {
    hipError_t e;
    if (cand) {
        e = hs::launch_zero_u64(cand_count, st);
        if (e != hipSuccess) return fail_hip(e, "counter reset");
    }
    hs::StatsArgs sa{};
    sa.x = x;
    sa.offsets = nullptr;
    sa.n_bins = n_bins;
    sa.rows = 1;
    sa.row_len = n_bins;
    sa.stride = n_bins;
    sa.first_bin = p->desc.first_bin;
    sa.chunks = hs::kChunksBatched;
    sa.user_norm = norm;
    sa.user_table_h = norm && p->desc.norm_kind == HS_NORM_TABLE ? p->desc.harmonics : 0;
    sa.il_spectra = n_spectra;
    sa.tab_t = p->tab_t;
    sa.tab_stride = p->max_groups;
    hs_status s = run_norm(p, sa, n_spectra, st);
    if (s != HS_OK) return s;
    hs::IlArgs a{};
    a.x = x;
    a.n_bins = n_bins;
    a.n_spectra = n_spectra;
    a.norm = p->norm;
    a.tab_t = p->tab_t;
    a.tab_stride = p->max_groups;
    a.first_bin = p->desc.first_bin;
    a.H = p->desc.harmonics;
    a.n_end = n_end_of(p->desc, n_bins);
    a.kmask = eligible_mask(p->desc);
    a.snr = snr;
    a.harm = harm;
    a.drift = drift;
    a.cand = cand;
    a.cap = cand_capacity;
    a.count = cand_count;
    a.thr = p->desc.threshold;
    a.n_groups = (n_spectra + 63) / 64;
    a.tile = kIlTile;
    a.n_tasks = (int64_t)a.n_groups * ((n_bins + kIlTile - 1) / kIlTile);
    a.n_xcd = p->n_xcd;
    e = hs::launch_sum_il(a, p->hmax, p->desc.mode == HS_GREEDY, p->desc.dtype == HS_F16, st);
    if (e != hipSuccess) return fail_hip(e, "interleaved harmonic-sum kernel");
    return mark(p, 2, st);
}

uint64_t W(const void *ptr) { return (uint64_t)(uintptr_t)ptr; }

constexpr size_t kGraphCache = 8;   // captured argument sets kept per plan

hs_status release_graph(hs_plan::GraphEntry &g) {
    hipError_t e = hipEventSynchronize(g.done);
    if (e == hipSuccess) e = hipGraphExecDestroy(g.exec);
    if (e == hipSuccess) e = hipEventDestroy(g.done);
    return e == hipSuccess ? HS_OK : fail_hip(e, "graph release");
}

hs_status clear_graphs(hs_plan *p) {
    hs_status s = HS_OK;
    for (auto &g : p->graphs) {
        hs_status r = release_graph(g);
        if (s == HS_OK) s = r;
    }
    p->graphs.clear();
    return s;
}

// Record one call (body) into a new graph of the plan's cache.
template <class Body>
hs_status capture(hs_plan *p, std::vector<uint64_t> &&key, Body &body, hs_plan::GraphEntry **out) {
    hipError_t e;
    if (!p->cap_stream) {
        e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail_hip(e, "hipStreamCreateWithFlags");
    }
    if (p->graphs.size() >= kGraphCache) {
        size_t lru = 0;
        for (size_t i = 1; i < p->graphs.size(); ++i)
            if (p->graphs[i].last_use < p->graphs[lru].last_use) lru = i;
        hs_status s = release_graph(p->graphs[lru]);
        p->graphs.erase(p->graphs.begin() + lru);
        if (s != HS_OK) return s;
    }
    e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail_hip(e, "hipStreamBeginCapture");
    hs_status s = body(p->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &graph);
    if (s != HS_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return s != HS_OK ? s : fail_hip(e, "hipStreamEndCapture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail_hip(e, "hipGraphInstantiate");
    hipEvent_t done = nullptr;
    e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return fail_hip(e, "hipEventCreate");
    }
    p->graphs.push_back(hs_plan::GraphEntry{std::move(key), exec, done, 0});
    *out = &p->graphs.back();
    ++p->captures;
    return HS_OK;
}

// Run one validated sum call: directly, or (graph mode) as a replay of the
// graph captured for the same arguments.  Calls made while the caller's
// stream is itself capturing, and timed calls, run directly (a timed call on
// a capturing stream is refused: its events would time nothing).
template <class Body>
hs_status dispatch(hs_plan *p, std::vector<uint64_t> &&key, hipStream_t st, Body body) {
    int cur = -1;
    hipError_t de = hipGetDevice(&cur);
    if (de != hipSuccess) return fail_hip(de, "hipGetDevice");
    if (cur != p->device) return fail(HS_ERR_ARG, "the plan belongs to another device than the current one");
    if (!p->graph && !p->timing) return body(st);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return fail_hip(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) {
        if (p->timing) return fail(HS_ERR_ARG, "stage timing is enabled while the stream is capturing");
        return body(st);
    }
    if (p->timing) return body(st);
    hs_plan::GraphEntry *g = nullptr;
    for (auto &c : p->graphs)
        if (c.key == key) {
            g = &c;
            break;
        }
    if (g) {
        ++p->replays;
    } else {
        hs_status s = capture(p, std::move(key), body, &g);
        if (s != HS_OK) return s;
    }
    g->last_use = ++p->graph_clock;
    e = hipGraphLaunch(g->exec, st);
    if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
    e = hipEventRecord(g->done, st);
    if (e != hipSuccess) return fail_hip(e, "hipEventRecord");
    return HS_OK;
}

// Largest workgroups per CU of the persistent kernel with F fundamentals per
// lane: what its registers and LDS allow (compiled for at most 8 waves per
// SIMD, i.e. 8 workgroups of 256).
hs_status resident_limit(hs_plan *p, int F, int *per_cu) {
    hipError_t e = hs::xcd_resident_blocks(p->hmax, p->desc.mode == HS_GREEDY, p->desc.dtype == HS_F16, F, per_cu);
    if (e != hipSuccess) return fail_hip(e, "occupancy query");
    const int cap = 8;
    if (*per_cu > cap) *per_cu = cap;
    if (*per_cu < 1) *per_cu = 1;
    return HS_OK;
}

hs_status set_shape(hs_plan *p, int F, int wgs_per_cu) {
    if (F == 0) {   // the plain kernel for batches (AUTO plans)
        if (p->desc.kernel != HS_KERNEL_AUTO) return fail(HS_ERR_ARG, "the plan fixes its kernel");
        if (!p->batched_plain) {
            hs_status s = clear_graphs(p);
            if (s != HS_OK) return s;
        }
        p->batched_plain = true;
        return HS_OK;
    }
    if (F != 1 && F != 2 && F != 4) return fail(HS_ERR_ARG, "fundamentals per lane must be 0, 1, 2 or 4");
    int lim = 0;
    hs_status s = resident_limit(p, F, &lim);
    if (s != HS_OK) return s;
    if (wgs_per_cu < 1 || wgs_per_cu > lim) return fail(HS_ERR_ARG, "workgroups per CU out of range");
    if (F != p->xcd_f || wgs_per_cu * p->n_cu != p->xcd_blocks || p->batched_plain) {
        s = clear_graphs(p);   // captured launches hold the old shape
        if (s != HS_OK) return s;
    }
    p->batched_plain = false;
    p->xcd_f = F;
    p->xcd_blocks = wgs_per_cu * p->n_cu;
    return HS_OK;
}

// ---------------------------------------------------------------------------
// Launch-shape tuner of the persistent kernel.  Every shape gives the same
// results bit for bit; only the time differs.  A cache file holds one JSON
// object per line: {"key": "...", "fundamentals_per_lane": F,
// "workgroups_per_cu": W, "ms": t}.
// ---------------------------------------------------------------------------

std::string tune_key(hs_plan *p, int64_t total_bins, int32_t n_spectra, bool dense, bool cand) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
        arch = prop.gcnArchName;
        size_t c = arch.find(':');
        if (c != std::string::npos) arch.resize(c);
    } else {
        (void)hipGetLastError();
    }
    int lg = 0;
    while (lg < 62 && (1ll << (lg + 1)) <= total_bins) ++lg;
    int ls = 0;
    while (ls < 30 && (1 << (ls + 1)) <= n_spectra) ++ls;
    char buf[256];
    snprintf(buf, sizeof buf, "%s cu%d xcd%d h%d %s %s %s%s bins2^%d spectra2^%d", arch.c_str(), p->n_cu, p->n_xcd,
             p->hmax, p->desc.mode == HS_GREEDY ? "greedy" : "standard", p->desc.dtype == HS_F16 ? "f16" : "f32",
             dense ? "dense" : "", cand ? "+cand" : "", lg, ls);
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, int *F, int *Wg) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    const std::string pat = "\"key\": \"" + key + "\"";
    char line[1024];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, pat.c_str())) continue;
        const char *a = strstr(line, "\"fundamentals_per_lane\":");
        const char *b = strstr(line, "\"workgroups_per_cu\":");
        if (!a || !b) continue;
        *F = atoi(a + strlen("\"fundamentals_per_lane\":"));
        *Wg = atoi(b + strlen("\"workgroups_per_cu\":"));
        found = true;   // the last matching line wins
    }
    fclose(f);
    return found;
}

hs_status tune_batched(hs_plan *p, const void *x, const int64_t *offsets, int32_t n_spectra, const double *norm,
                       float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand, int64_t cand_capacity,
                       unsigned long long *cand_count, const char *cache_path, hipStream_t st) {
    if (p->desc.kernel == HS_KERNEL_PLAIN) return fail(HS_ERR_ARG, "the plan uses the plain kernel: nothing to tune");
    auto call = [&]() {
        return hs_sum_batched(p, x, offsets, n_spectra, norm, snr, harm, drift, cand, cand_capacity, cand_count,
                              (void *)st);
    };
    hs_status s = call();   // validates the arguments and warms up
    if (s != HS_OK) return s;
    int64_t total = 0;
    hipError_t e = hipMemcpyAsync(&total, offsets + n_spectra, sizeof total, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail_hip(e, "reading the batch size");
    const std::string key = tune_key(p, total, n_spectra, snr != nullptr, cand != nullptr);
    int F = 0, Wg = 0;
    if (cache_path && cache_lookup(cache_path, key, &F, &Wg) && set_shape(p, F, Wg) == HS_OK) return HS_OK;

    hipEvent_t t0 = nullptr, t1 = nullptr;
    e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        return fail_hip(e, "hipEventCreate");
    }
    const int F0 = p->batched_plain ? 0 : p->xcd_f, W0 = p->batched_plain ? 0 : p->xcd_blocks / p->n_cu;
    int bestF = F0, bestW = W0;
    float best = 3.4e38f;
    for (int f : {0, 1, 2, 4}) {
        if (f == 0 && p->desc.kernel != HS_KERNEL_AUTO) continue;
        int lim = 0;   // the plain kernel has one shape
        if (f != 0) s = resident_limit(p, f, &lim);
        if (s != HS_OK) break;
        for (int w = f == 0 ? 0 : 1; w <= lim && s == HS_OK; ++w) {
            s = set_shape(p, f, w);
            if (s == HS_OK) s = call();   // warm-up of this shape
            float t[3];
            for (int r = 0; r < 3 && s == HS_OK; ++r) {
                e = hipEventRecord(t0, st);
                if (e != hipSuccess) {
                    s = fail_hip(e, "hipEventRecord");
                    break;
                }
                s = call();
                if (s != HS_OK) break;
                e = hipEventRecord(t1, st);
                if (e == hipSuccess) e = hipEventSynchronize(t1);
                if (e == hipSuccess) e = hipEventElapsedTime(&t[r], t0, t1);
                if (e != hipSuccess) s = fail_hip(e, "timing a tuning run");
            }
            if (s != HS_OK) break;
            float med = t[0] < t[1] ? (t[1] < t[2] ? t[1] : (t[0] < t[2] ? t[2] : t[0]))
                                    : (t[0] < t[2] ? t[0] : (t[1] < t[2] ? t[2] : t[1]));
            if (med < best) {
                best = med;
                bestF = f;
                bestW = w;
            }
        }
        if (s != HS_OK) break;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (s != HS_OK) {
        (void)set_shape(p, F0, W0);
        return s;
    }
    s = set_shape(p, bestF, bestW);
    if (s != HS_OK) return s;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (!f) return fail(HS_ERR_ARG, "cannot append to the tuning cache file");
        fprintf(f, "{\"key\": \"%s\", \"fundamentals_per_lane\": %d, \"workgroups_per_cu\": %d, \"ms\": %.4f}\n",
                key.c_str(), bestF, bestW, best);
        fclose(f);
    }
    return HS_OK;
}

hs_status check_desc(const hs_plan_desc &d) {
    if (d.harmonics < 1) return fail(HS_ERR_ARG, "harmonics must be >= 1");
    if (d.harmonics > HS_MAX_HARMONICS) return fail(HS_ERR_UNSUPPORTED, "harmonics above 64 not supported");
    if (is_presto(d.mode) && d.harmonics > 32)
        return fail(HS_ERR_UNSUPPORTED, "the PRESTO-style sums support harmonics up to 32");
    if (d.norm_kind != HS_NORM_MU_SIGMA && d.norm_kind != HS_NORM_TABLE) return fail(HS_ERR_ARG, "bad norm_kind");
    if (d.mode != HS_STANDARD && d.mode != HS_GREEDY && !is_presto(d.mode)) return fail(HS_ERR_ARG, "bad mode");
    if (d.dtype != HS_F32 && d.dtype != HS_F16) return fail(HS_ERR_ARG, "bad dtype");
    if (d.first_bin < 1) return fail(HS_ERR_ARG, "first_bin must be >= 1");
    if (d.fundamental_end < 0) return fail(HS_ERR_ARG, "fundamental_end must be >= 0");
    if (d.max_spectra < 1 || d.max_spectra > 65535) return fail(HS_ERR_ARG, "max_spectra out of range [1, 65535]");
    if (d.harmonics < 64 && (d.report_mask >> d.harmonics) != 0) return fail(HS_ERR_ARG, "report_mask above H");
    if (d.harmonic_mask != 0 && eligible_mask(d) == 0) return fail(HS_ERR_ARG, "harmonic_mask selects no k <= H");
    if (!(d.threshold == d.threshold)) return fail(HS_ERR_ARG, "threshold is NaN");
    if (d.kernel < HS_KERNEL_AUTO || d.kernel > HS_KERNEL_PLAIN) return fail(HS_ERR_ARG, "bad kernel choice");
    if (is_presto(d.mode) && d.report_mask != 0)
        return fail(HS_ERR_UNSUPPORTED, "partial sums are reported for the simple and greedy sums only");
    if (is_presto(d.mode) && d.kernel == HS_KERNEL_PERSISTENT)
        return fail(HS_ERR_UNSUPPORTED, "the PRESTO-style sums have one kernel (AUTO or PLAIN)");
    return HS_OK;
}

// Device workspace of a plan: one block, pieces at 256-byte aligned offsets.
struct Layout {
    int parts_cap;
    size_t norm, parts, tickets, prefix, ray, tab_t, total;
};

constexpr size_t kWsAlign = 256;

size_t align_up(size_t v) { return (v + kWsAlign - 1) & ~(kWsAlign - 1); }

Layout layout(const hs_plan_desc &d) {
    Layout l{};
    int64_t parts = (int64_t)d.max_spectra * hs::kChunksBatched;
    if (parts < hs::kChunks2D) parts = hs::kChunks2D;
    if (parts < hs::kChunks1D) parts = hs::kChunks1D;
    l.parts_cap = (int)parts;
    size_t o = 0;
    l.norm = o;
    o = align_up(o + sizeof(hs::NormRec) * (size_t)d.max_spectra);
    l.parts = o;
    o = align_up(o + sizeof(hs::StatPart) * (size_t)l.parts_cap);
    l.tickets = o;
    o = align_up(o + sizeof(uint32_t) * hs::kMaxXcd);
    l.prefix = o;
    o = align_up(o + sizeof(uint32_t) * ((size_t)d.max_spectra + 1));
    l.ray = o;
    o = align_up(o + sizeof(hs::RayBand) * hs::kRayMaxBands);
    l.tab_t = o;
    o = align_up(o + sizeof(float2) * HS_MAX_HARMONICS * (size_t)d.max_spectra);
    l.total = o;
    return l;
}

// Plan on the current device; workspace == NULL: the plan allocates (and
// later frees) its workspace, else it uses the caller's.
hs_status create_plan(const hs_plan_desc *desc, void *workspace, size_t bytes, hs_plan **plan) {
    if (!desc || !plan) return fail(HS_ERR_ARG, "null argument");
    *plan = nullptr;
    const hs_plan_desc &d = *desc;
    hs_status cs = check_desc(d);
    if (cs != HS_OK) return cs;
    const Layout l = layout(d);
    if (workspace) {
        if (((uintptr_t)workspace & (kWsAlign - 1)) != 0) return fail(HS_ERR_ARG, "workspace not 256-byte aligned");
        if (bytes < l.total) return fail(HS_ERR_ARG, "workspace smaller than hs_plan_workspace_bytes");
    }
    hs_plan *p = new (std::nothrow) hs_plan();
    if (!p) return fail(HS_ERR_NOMEM, "host allocation failed");
    p->desc = d;
    p->hmax = bucket(d.harmonics);
    p->max_groups = d.max_spectra;
    p->parts_cap = l.parts_cap;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "hipGetDevice");
    }
    if (workspace) {
        p->ws = (char *)workspace;
        p->ws_owned = false;
    } else {
        e = hipMalloc((void **)&p->ws, l.total);
        if (e != hipSuccess) {
            delete p;
            (void)hipGetLastError();
            return fail(HS_ERR_NOMEM, "device workspace allocation failed");
        }
        p->ws_owned = true;
    }
    p->norm = (hs::NormRec *)(p->ws + l.norm);
    p->parts = (hs::StatPart *)(p->ws + l.parts);
    p->tickets = (uint32_t *)(p->ws + l.tickets);
    p->prefix = (uint32_t *)(p->ws + l.prefix);
    p->ray = (hs::RayBand *)(p->ws + l.ray);
    p->tab_t = (float2 *)(p->ws + l.tab_t);
    hs_status ss = setup_xcd(p);
    if (ss != HS_OK) {
        hs_plan_destroy(p);
        return ss;
    }
    *plan = p;
    return HS_OK;
}

// Allocation-free batched sum: the workspace of hs_sum_batched_static is this
// file-scope device array instead of a plan's hipMalloc.  Each device holds
// its own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns on that device (the array's name is a
// host-side stand-in).
constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr int kScratchMaxSpectra = 1024;
constexpr int kScratchDevices = 64;
__device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu;
char *g_scratch_ptr[kScratchDevices];

// The device address of `scratch` on device dev (current), looked up once.
hs_status scratch_of(int dev, char **out) {
    if (dev < 0 || dev >= kScratchDevices) return fail(HS_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = (char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return HS_OK;
}

}  // namespace

extern "C" {

void hs_plan_desc_init(hs_plan_desc *d) {
    if (!d) return;
    memset(d, 0, sizeof(*d));
    d->harmonics = 32;
    d->mode = HS_GREEDY;
    d->dtype = HS_F32;
    d->first_bin = 1;
    d->harmonic_mask = 0;
    d->report_mask = 0;
    d->fundamental_end = 0;
    d->max_spectra = 1024;
    d->threshold = 6.0f;
    d->kernel = HS_KERNEL_AUTO;
    d->norm_kind = HS_NORM_MU_SIGMA;
}

hs_status hs_plan_workspace_bytes(const hs_plan_desc *desc, size_t *bytes) {
    return guarded([&]() -> hs_status {
        if (!desc || !bytes) return fail(HS_ERR_ARG, "null argument");
        hs_status s = check_desc(*desc);
        if (s != HS_OK) return s;
        *bytes = layout(*desc).total;
        return HS_OK;
    });
}

hs_status hs_plan_create(const hs_plan_desc *desc, hs_plan **plan) {
    return guarded([&]() -> hs_status {
        return create_plan(desc, nullptr, 0, plan);
    });
}

hs_status hs_plan_create_in(const hs_plan_desc *desc, void *workspace, size_t bytes, hs_plan **plan) {
    return guarded([&]() -> hs_status {
        if (!workspace) return fail(HS_ERR_ARG, "null workspace");
        return create_plan(desc, workspace, bytes, plan);
    });
}

hs_status hs_plan_destroy(hs_plan *p) {
    return guarded([&]() -> hs_status {
        if (!p) return fail(HS_ERR_ARG, "null plan");
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p->device);
        if (p->ws_owned) (void)hipFree(p->ws);
        for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
        (void)clear_graphs(p);
        if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
        (void)hipSetDevice(cur);
        delete p;
        return HS_OK;
    });
}

hs_status hs_sum_1d(hs_plan *p, const void *x, int64_t n_bins, const double *norm, float *snr, uint8_t *harm,
                    uint8_t *drift, float *partial, void *stream) {
    return guarded([&]() -> hs_status {
        if (!p || !x || !snr || !harm) return fail(HS_ERR_ARG, "null argument");
        if (!norm && p->desc.norm_kind == HS_NORM_TABLE) return fail(HS_ERR_ARG, "HS_NORM_TABLE needs the norm table");
        if (n_bins < 2 || n_bins >= (1ll << 30)) return fail(HS_ERR_ARG, "n_bins out of range [2, 2^30)");
        if (!aligned_elem(x, p->desc.dtype)) return fail(HS_ERR_ARG, "x must be aligned to its element size");
        if (p->desc.report_mask != 0 && !partial) return fail(HS_ERR_ARG, "report_mask set but partial is NULL");
        hipStream_t st = (hipStream_t)stream;
        return dispatch(p, {1, W(x), (uint64_t)n_bins, W(norm), W(snr), W(harm), W(drift), W(partial)}, st,
                        [=](hipStream_t s) { return enqueue_1d(p, x, n_bins, norm, snr, harm, drift, partial, s); });
    });
}

hs_status hs_sum_batched(hs_plan *p, const void *x, const int64_t *offsets, int32_t n_spectra, const double *norm,
                         float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand, int64_t cand_capacity,
                         unsigned long long *cand_count, void *stream) {
    return guarded([&]() -> hs_status {
        if (!p || !x || !offsets) return fail(HS_ERR_ARG, "null argument");
        if (!norm && p->desc.norm_kind == HS_NORM_TABLE) return fail(HS_ERR_ARG, "HS_NORM_TABLE needs the norm table");
        if (n_spectra < 1 || n_spectra > p->max_groups) return fail(HS_ERR_ARG, "n_spectra out of range");
        if (!aligned_elem(x, p->desc.dtype)) return fail(HS_ERR_ARG, "x must be aligned to its element size");
        if (!snr && !cand) return fail(HS_ERR_ARG, "neither dense outputs nor candidates requested");
        if (snr && !harm) return fail(HS_ERR_ARG, "snr given without harm");
        if (cand && (!cand_count || cand_capacity < 0)) return fail(HS_ERR_ARG, "candidate buffer needs a counter");
        hipStream_t st = (hipStream_t)stream;
        return dispatch(p,
                        {2, W(x), W(offsets), (uint64_t)n_spectra, W(norm), W(snr), W(harm), W(drift), W(cand),
                         (uint64_t)cand_capacity, W(cand_count)},
                        st, [=](hipStream_t s) {
                            return enqueue_batched(p, x, offsets, n_spectra, norm, snr, harm, drift, cand, cand_capacity,
                                                   cand_count, s);
                        });
    });
}

hs_status hs_sum_2d(hs_plan *p, const void *plane, int64_t n_r, int64_t row_stride, int32_t z_min, int32_t z_max,
                    const double *norm, float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand,
                    int64_t cand_capacity, unsigned long long *cand_count, void *stream) {
    return guarded([&]() -> hs_status {
        if (!p || !plane) return fail(HS_ERR_ARG, "null argument");
        if (!norm && p->desc.norm_kind == HS_NORM_TABLE) return fail(HS_ERR_ARG, "HS_NORM_TABLE needs the norm table");
        if (is_presto(p->desc.mode)) return fail(HS_ERR_UNSUPPORTED, "no f-fdot form of the PRESTO-style sums");
        if (n_r < 2 || n_r >= (1ll << 30)) return fail(HS_ERR_ARG, "n_r out of range [2, 2^30)");
        if (row_stride < n_r) return fail(HS_ERR_ARG, "row_stride < n_r");
        if (z_max < z_min) return fail(HS_ERR_ARG, "z_max < z_min");
        const int64_t n_z = (int64_t)z_max - z_min + 1;
        if (n_z > 65535) return fail(HS_ERR_UNSUPPORTED, "more than 65535 rows");
        if (!aligned_elem(plane, p->desc.dtype)) return fail(HS_ERR_ARG, "plane must be aligned to its element size");
        if (!snr && !cand) return fail(HS_ERR_ARG, "neither dense outputs nor candidates requested");
        if (snr && !harm) return fail(HS_ERR_ARG, "snr given without harm");
        if (cand && (!cand_count || cand_capacity < 0)) return fail(HS_ERR_ARG, "candidate buffer needs a counter");
        if (cand && n_z * n_r > 0xffffffffll) return fail(HS_ERR_UNSUPPORTED, "plane too large for 32-bit candidate bins");
        hipStream_t st = (hipStream_t)stream;
        return dispatch(p,
                        {3, W(plane), (uint64_t)n_r, (uint64_t)row_stride, (uint64_t)(uint32_t)z_min,
                         (uint64_t)(uint32_t)z_max, W(norm), W(snr), W(harm), W(drift), W(cand), (uint64_t)cand_capacity,
                         W(cand_count)},
                        st, [=](hipStream_t s) {
                            return enqueue_2d(p, plane, n_r, row_stride, z_min, z_max, norm, snr, harm, drift, cand,
                                              cand_capacity, cand_count, s);
                        });
    });
}

hs_status hs_sum_interleaved(hs_plan *p, const void *x, int64_t n_bins, int32_t n_spectra, const double *norm,
                             float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand, int64_t cand_capacity,
                             unsigned long long *cand_count, void *stream) {
    return guarded([&]() -> hs_status {
        if (!p || !x) return fail(HS_ERR_ARG, "null argument");
        if (p->desc.mode != HS_STANDARD && p->desc.mode != HS_GREEDY)
            return fail(HS_ERR_UNSUPPORTED, "the interleaved layout runs the simple and greedy sums");
        if (!norm && p->desc.norm_kind == HS_NORM_TABLE) return fail(HS_ERR_ARG, "HS_NORM_TABLE needs the norm table");
        if (n_spectra < 1 || n_spectra > p->max_groups) return fail(HS_ERR_ARG, "n_spectra out of range");
        if (n_bins < 2 || n_bins * (int64_t)n_spectra >= (1ll << 30))
            return fail(HS_ERR_ARG, "n_bins out of range [2, 2^30 / n_spectra)");
        if (!aligned_elem(x, p->desc.dtype)) return fail(HS_ERR_ARG, "x must be aligned to its element size");
        if (!snr && !cand) return fail(HS_ERR_ARG, "neither dense outputs nor candidates requested");
        if (snr && !harm) return fail(HS_ERR_ARG, "snr given without harm");
        if (cand && (!cand_count || cand_capacity < 0)) return fail(HS_ERR_ARG, "candidate buffer needs a counter");
        hipStream_t st = (hipStream_t)stream;
        return dispatch(p,
                        {4, W(x), (uint64_t)n_bins, (uint64_t)n_spectra, W(norm), W(snr), W(harm), W(drift), W(cand),
                         (uint64_t)cand_capacity, W(cand_count)},
                        st, [=](hipStream_t s) {
                            return enqueue_interleaved(p, x, n_bins, n_spectra, norm, snr, harm, drift, cand,
                                                       cand_capacity, cand_count, s);
                        });
    });
}

hs_status hs_interleave(const void *x, int64_t n_bins, int32_t n_spectra, int32_t elem_bytes, void *out,
                        void *stream) {
    return guarded([&]() -> hs_status {
        if (!x || !out) return fail(HS_ERR_ARG, "null argument");
        if (elem_bytes != 2 && elem_bytes != 4) return fail(HS_ERR_ARG, "elem_bytes must be 2 or 4");
        if (n_bins < 1 || n_spectra < 1 || n_spectra > 65535 * 64 || (n_bins + 63) / 64 > 0x7fffffffll)
            return fail(HS_ERR_ARG, "sizes out of range");
        if (((uintptr_t)x | (uintptr_t)out) & (uintptr_t)(elem_bytes - 1)) return fail(HS_ERR_ARG, "misaligned buffer");
        const char *xb = (const char *)x, *ob = (const char *)out;
        const int64_t bytes = n_bins * n_spectra * (int64_t)elem_bytes;
        if (xb < ob + bytes && ob < xb + bytes) return fail(HS_ERR_ARG, "x and out overlap");
        hipError_t e = hs::launch_interleave(x, n_bins, n_spectra, elem_bytes, out, (hipStream_t)stream);
        if (e != hipSuccess) return fail_hip(e, "interleave kernel");
        return HS_OK;
    });
}

hs_status hs_power_spectrum(const void *fft, int64_t n_bins, int32_t interbin, float scale, float *out, void *stream) {
    return guarded([&]() -> hs_status {
        if (!fft || !out) return fail(HS_ERR_ARG, "null argument");
        if (n_bins < 1 || n_bins >= (1ll << 31)) return fail(HS_ERR_ARG, "n_bins out of range [1, 2^31)");
        if (((uintptr_t)fft & 7u) || ((uintptr_t)out & 3u)) return fail(HS_ERR_ARG, "misaligned buffer");
        if (!(scale > 0.0f) || !(scale < __builtin_inff())) return fail(HS_ERR_ARG, "scale must be positive and finite");
        const int64_t out_n = interbin ? 2 * n_bins - 1 : n_bins;
        const char *a = (const char *)fft, *b = (const char *)out;
        if (a < b + 4 * out_n && b < a + 8 * n_bins) return fail(HS_ERR_ARG, "fft and out overlap");
        // scale (pi/4)^2: the float factor rounded once, times scale in double, rounded once
        const float f16 = (float)((M_PI * M_PI) / 16.0);
        const float sch = (float)((double)scale * (double)f16);
        hipError_t e = hs::launch_power(fft, n_bins, interbin != 0, scale, sch, out, (hipStream_t)stream);
        if (e != hipSuccess) return fail_hip(e, "power-spectrum kernel");
        return HS_OK;
    });
}

hs_status hs_cluster_peaks(const float *snr, const uint8_t *harm, const uint8_t *drift, const int64_t *offsets,
                           int64_t n_bins, int32_t n_spectra, int32_t radius, float threshold, hs_candidate *cand,
                           int64_t cand_capacity, unsigned long long *cand_count, void *stream) {
    return guarded([&]() -> hs_status {
        if (!snr || !harm || !cand_count || (!cand && cand_capacity > 0)) return fail(HS_ERR_ARG, "null argument");
        if (cand_capacity < 0) return fail(HS_ERR_ARG, "negative capacity");
        if (n_bins < 1 || n_bins >= (1ll << 32)) return fail(HS_ERR_ARG, "n_bins out of range [1, 2^32)");
        if (offsets ? (n_spectra < 1 || n_spectra > 65535) : n_spectra != 1) return fail(HS_ERR_ARG, "n_spectra out of range");
        if (radius < 0) return fail(HS_ERR_ARG, "radius < 0");
        if (!(threshold == threshold)) return fail(HS_ERR_ARG, "threshold is NaN");
        if (((uintptr_t)snr & 3u)) return fail(HS_ERR_ARG, "misaligned snr");
        hipStream_t st = (hipStream_t)stream;
        hipError_t e = hs::launch_zero_u64(cand_count, st);
        if (e != hipSuccess) return fail_hip(e, "counter reset");
        hs::PeakArgs a{};
        a.snr = snr;
        a.harm = harm;
        a.drift = drift;
        a.offsets = offsets;
        a.n_bins = n_bins;
        a.radius = radius;
        a.thr = threshold;
        a.cand = cand;
        a.cap = cand_capacity;
        a.count = cand_count;
        e = hs::launch_peaks(a, offsets ? n_spectra : 1, offsets ? (n_bins + n_spectra - 1) / n_spectra : n_bins, st);
        if (e != hipSuccess) return fail_hip(e, "peak kernel");
        return HS_OK;
    });
}

hs_status hs_get_norm(hs_plan *p, int32_t n, double *mu_sigma, float *tables, int32_t *valid, void *stream) {
    return guarded([&]() -> hs_status {
        if (!p) return fail(HS_ERR_ARG, "null plan");
        if (n < 1 || n > p->last_groups) return fail(HS_ERR_ARG, "n exceeds the groups of the last call");
        if (!mu_sigma && !tables && !valid) return fail(HS_ERR_ARG, "nothing to export");
        hipError_t e = hs::launch_export_norm(p->norm, n, p->desc.harmonics, mu_sigma, tables, valid,
                                              (hipStream_t)stream);
        if (e != hipSuccess) return fail_hip(e, "export kernel");
        return HS_OK;
    });
}

hs_status hs_quantize_f16(const float *x, int64_t n, float scale, uint16_t *out, void *stream) {
    return guarded([&]() -> hs_status {
        if (!x || !out) return fail(HS_ERR_ARG, "null argument");
        if (n < 0) return fail(HS_ERR_ARG, "n < 0");
        if (!(scale > 0.0f) || !(scale < __builtin_inff())) return fail(HS_ERR_ARG, "scale must be positive and finite");
        if (n == 0) return HS_OK;
        hipError_t e = hs::launch_quantize_f16(x, n, scale, out, (hipStream_t)stream);
        if (e != hipSuccess) return fail_hip(e, "quantise kernel");
        return HS_OK;
    });
}

hs_status hs_plan_set_timing(hs_plan *p, int32_t enable) {
    return guarded([&]() -> hs_status {
        if (!p) return fail(HS_ERR_ARG, "null plan");
        p->timing = enable != 0;
        p->ev_used = 0;
        return HS_OK;
    });
}

hs_status hs_plan_get_timing(hs_plan *p, int32_t *calls, double *norm_ms, double *sum_ms) {
    return guarded([&]() -> hs_status {
        if (!p) return fail(HS_ERR_ARG, "null plan");
        double a = 0.0, b = 0.0;
        for (int i = 0; i + 2 < p->ev_used; i += 3) {
            hipError_t e = hipEventSynchronize(p->ev[i + 2]);
            if (e != hipSuccess) return fail_hip(e, "hipEventSynchronize");
            float t01 = 0.0f, t12 = 0.0f;
            e = hipEventElapsedTime(&t01, p->ev[i], p->ev[i + 1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&t12, p->ev[i + 1], p->ev[i + 2]);
            if (e != hipSuccess) return fail_hip(e, "hipEventElapsedTime");
            a += t01;
            b += t12;
        }
        if (calls) *calls = p->ev_used / 3;
        if (norm_ms) *norm_ms = a;
        if (sum_ms) *sum_ms = b;
        p->ev_used = 0;
        return HS_OK;
    });
}

hs_status hs_plan_set_graph(hs_plan *p, int32_t enable) {
    return guarded([&]() -> hs_status {
        if (!p) return fail(HS_ERR_ARG, "null plan");
        p->graph = enable != 0;
        return p->graph ? HS_OK : clear_graphs(p);
    });
}

hs_status hs_plan_graph_info(hs_plan *p, int64_t *captures, int64_t *replays) {
    return guarded([&]() -> hs_status {
        if (!p) return fail(HS_ERR_ARG, "null plan");
        if (captures) *captures = p->captures;
        if (replays) *replays = p->replays;
        return HS_OK;
    });
}

hs_status hs_plan_set_launch(hs_plan *p, int32_t fundamentals_per_lane, int32_t workgroups_per_cu) {
    return guarded([&]() -> hs_status {
        if (!p) return fail(HS_ERR_ARG, "null plan");
        if (is_presto(p->desc.mode)) return fail(HS_ERR_UNSUPPORTED, "the PRESTO-style sums have no launch shape");
        return set_shape(p, fundamentals_per_lane, workgroups_per_cu);
    });
}

hs_status hs_plan_get_launch(hs_plan *p, int32_t *fundamentals_per_lane, int32_t *workgroups_per_cu) {
    return guarded([&]() -> hs_status {
        if (!p) return fail(HS_ERR_ARG, "null plan");
        if (fundamentals_per_lane) *fundamentals_per_lane = p->batched_plain ? 0 : p->xcd_f;
        if (workgroups_per_cu) *workgroups_per_cu = p->batched_plain ? 0 : p->xcd_blocks / p->n_cu;
        return HS_OK;
    });
}

hs_status hs_plan_tune_batched(hs_plan *p, const void *x, const int64_t *offsets, int32_t n_spectra,
                               const double *norm, float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand,
                               int64_t cand_capacity, unsigned long long *cand_count, const char *cache_path,
                               void *stream) {
    return guarded([&]() -> hs_status {
        if (!p) return fail(HS_ERR_ARG, "null plan");
        if (is_presto(p->desc.mode)) return fail(HS_ERR_UNSUPPORTED, "the PRESTO-style sums have no launch shape");
        if (p->timing) return fail(HS_ERR_ARG, "stage timing is enabled");
        hipStream_t st = (hipStream_t)stream;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(st, &cs);
        if (e != hipSuccess) return fail_hip(e, "hipStreamIsCapturing");
        if (cs != hipStreamCaptureStatusNone) return fail(HS_ERR_ARG, "the stream is capturing");
        const bool graph = p->graph;
        p->graph = false;
        hs_status s = tune_batched(p, x, offsets, n_spectra, norm, snr, harm, drift, cand, cand_capacity, cand_count,
                                   cache_path, st);
        p->graph = graph;
        return s;
    });
}

hs_status hs_sum_batched_static(const hs_plan_desc *desc, const void *x, const int64_t *offsets, int32_t n_spectra,
                                const double *norm, float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand,
                                int64_t cand_capacity, unsigned long long *cand_count, void *stream) {
    return guarded([&]() -> hs_status {
        if (!desc || !x || !offsets) return fail(HS_ERR_ARG, "null argument");
        hs_status cs = check_desc(*desc);
        if (cs != HS_OK) return cs;
        if (!norm && desc->norm_kind == HS_NORM_TABLE) return fail(HS_ERR_ARG, "HS_NORM_TABLE needs the norm table");
        if (n_spectra < 1 || n_spectra > kScratchMaxSpectra)
            return fail(HS_ERR_ARG, "n_spectra out of range [1, 1024] of the allocation-free call");
        if (!aligned_elem(x, desc->dtype)) return fail(HS_ERR_ARG, "x must be aligned to its element size");
        if (!snr && !cand) return fail(HS_ERR_ARG, "neither dense outputs nor candidates requested");
        if (snr && !harm) return fail(HS_ERR_ARG, "snr given without harm");
        if (cand && (!cand_count || cand_capacity < 0)) return fail(HS_ERR_ARG, "candidate buffer needs a counter");
        hs_plan_desc d = *desc;
        d.max_spectra = n_spectra;
        const Layout l = layout(d);
        if (l.total > kScratchBytes) return fail(HS_ERR_ARG, "workspace of this call exceeds the 4 MiB scratch");
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
        char *ws = nullptr;
        hs_status s = scratch_of(dev, &ws);
        if (s != HS_OK) return s;
        hs_plan p{};                     // on the stack: no graph cache, no timing events, nothing allocated
        p.desc = d;
        p.device = dev;
        p.hmax = bucket(d.harmonics);
        p.max_groups = n_spectra;
        p.parts_cap = l.parts_cap;
        p.ws = ws;
        p.ws_owned = false;
        p.norm = (hs::NormRec *)(ws + l.norm);
        p.parts = (hs::StatPart *)(ws + l.parts);
        p.tickets = (uint32_t *)(ws + l.tickets);
        p.prefix = (uint32_t *)(ws + l.prefix);
        p.ray = (hs::RayBand *)(ws + l.ray);
        p.tab_t = (float2 *)(ws + l.tab_t);
        s = setup_xcd(&p);
        if (s != HS_OK) return s;
        return enqueue_batched(&p, x, offsets, n_spectra, norm, snr, harm, drift, cand, cand_capacity, cand_count,
                               (hipStream_t)stream);
    });
}

const char *hs_status_string(hs_status s) {
    switch (s) {
        case HS_OK: return "ok";
        case HS_ERR_ARG: return "invalid argument";
        case HS_ERR_UNSUPPORTED: return "unsupported";
        case HS_ERR_HIP: return "HIP runtime error";
        case HS_ERR_NOMEM: return "out of memory";
        case HS_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *hs_last_error(void) { return g_last_error; }

}  // extern "C"
