// C ABI of the harmonic-sum library: argument validation, plan/workspace
// management and the launch sequence of every entry point (declared and
// documented in include/hs.h).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <string>

#include "hs_internal.h"

namespace {

thread_local std::string g_last_error;

hs_status fail(hs_status s, const char *msg) {
    g_last_error = msg;
    return s;
}

hs_status fail_hip(hipError_t e, const char *where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return HS_ERR_HIP;
}

int bucket(int H) {
    if (H <= 4) return 4;
    if (H <= 8) return 8;
    if (H <= 16) return 16;
    return 32;
}

// natural alignment of the stored powers
bool aligned_elem(const void *p, int dtype) { return ((uintptr_t)p & (dtype == HS_F16 ? 1u : 3u)) == 0; }

uint64_t eligible_mask(const hs_plan_desc &d) {
    const uint64_t all = d.harmonics >= 64 ? ~0ull : ((1ull << d.harmonics) - 1ull);
    return d.harmonic_mask ? (d.harmonic_mask & all) : all;
}

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
        e = hs::launch_stats(sa, groups, p->desc.dtype == HS_F16, st);
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
    int F = env_int("HS_XCD_F", 4);
    p->xcd_f = (F == 2 || F == 4) ? F : 4;
    int per_cu = 0;
    e = hs::xcd_resident_blocks(p->hmax, p->desc.mode == HS_GREEDY, p->desc.dtype == HS_F16, p->xcd_f, &per_cu);
    if (e != hipSuccess) return fail_hip(e, "occupancy query");
    // at most 4 resident workgroups per CU (the kernel is compiled for <= 4 waves
    // per SIMD so that it never spills); measured fastest at 4 for FP32 and FP16
    int want = env_int("HS_XCD_WGS_PER_CU", p->desc.dtype == HS_F16 ? per_cu : 4);
    if (want >= 1 && want < per_cu) per_cu = want;
    if (per_cu < 1) per_cu = 1;
    p->xcd_blocks = per_cu * p->n_cu;
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
}

hs_status hs_plan_create(const hs_plan_desc *desc, hs_plan **plan) {
    if (!desc || !plan) return fail(HS_ERR_ARG, "null argument");
    *plan = nullptr;
    const hs_plan_desc &d = *desc;
    if (d.harmonics < 1) return fail(HS_ERR_ARG, "harmonics must be >= 1");
    if (d.harmonics > HS_MAX_HARMONICS) return fail(HS_ERR_UNSUPPORTED, "harmonics above 32 not supported");
    if (d.mode != HS_STANDARD && d.mode != HS_GREEDY) return fail(HS_ERR_ARG, "bad mode");
    if (d.dtype != HS_F32 && d.dtype != HS_F16) return fail(HS_ERR_ARG, "bad dtype");
    if (d.first_bin < 1) return fail(HS_ERR_ARG, "first_bin must be >= 1");
    if (d.fundamental_end < 0) return fail(HS_ERR_ARG, "fundamental_end must be >= 0");
    if (d.max_spectra < 1 || d.max_spectra > 65535) return fail(HS_ERR_ARG, "max_spectra out of range [1, 65535]");
    if (d.harmonics < 64 && (d.report_mask >> d.harmonics) != 0) return fail(HS_ERR_ARG, "report_mask above H");
    if (d.harmonic_mask != 0 && eligible_mask(d) == 0) return fail(HS_ERR_ARG, "harmonic_mask selects no k <= H");
    if (!(d.threshold == d.threshold)) return fail(HS_ERR_ARG, "threshold is NaN");
    if (d.kernel < HS_KERNEL_AUTO || d.kernel > HS_KERNEL_PLAIN) return fail(HS_ERR_ARG, "bad kernel choice");

    hs_plan *p = new (std::nothrow) hs_plan();
    if (!p) return fail(HS_ERR_NOMEM, "host allocation failed");
    p->desc = d;
    p->hmax = bucket(d.harmonics);
    p->max_groups = d.max_spectra;
    int64_t parts = (int64_t)d.max_spectra * hs::kChunksBatched;
    if (parts < hs::kChunks2D) parts = hs::kChunks2D;
    if (parts < hs::kChunks1D) parts = hs::kChunks1D;
    p->parts_cap = (int)parts;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "hipGetDevice");
    }
    e = hipMalloc((void **)&p->norm, sizeof(hs::NormRec) * (size_t)p->max_groups);
    if (e == hipSuccess) e = hipMalloc((void **)&p->parts, sizeof(hs::StatPart) * (size_t)p->parts_cap);
    if (e == hipSuccess) e = hipMalloc((void **)&p->tickets, sizeof(uint32_t) * hs::kMaxXcd);
    if (e == hipSuccess) e = hipMalloc((void **)&p->prefix, sizeof(uint32_t) * ((size_t)p->max_groups + 1));
    if (e != hipSuccess) {
        if (p->norm) (void)hipFree(p->norm);
        if (p->parts) (void)hipFree(p->parts);
        if (p->tickets) (void)hipFree(p->tickets);
        delete p;
        (void)hipGetLastError();
        return fail(HS_ERR_NOMEM, "device workspace allocation failed");
    }
    hs_status ss = setup_xcd(p);
    if (ss != HS_OK) {
        hs_plan_destroy(p);
        return ss;
    }
    *plan = p;
    return HS_OK;
}

hs_status hs_plan_destroy(hs_plan *p) {
    if (!p) return fail(HS_ERR_ARG, "null plan");
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    (void)hipFree(p->norm);
    (void)hipFree(p->parts);
    (void)hipFree(p->tickets);
    (void)hipFree(p->prefix);
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    (void)hipSetDevice(cur);
    delete p;
    return HS_OK;
}

hs_status hs_sum_1d(hs_plan *p, const void *x, int64_t n_bins, const double *norm, float *snr, uint8_t *harm,
                    uint8_t *drift, float *partial, void *stream) {
    if (!p || !x || !snr || !harm) return fail(HS_ERR_ARG, "null argument");
    if (n_bins < 2 || n_bins >= (1ll << 30)) return fail(HS_ERR_ARG, "n_bins out of range [2, 2^30)");
    if (!aligned_elem(x, p->desc.dtype)) return fail(HS_ERR_ARG, "x must be aligned to its element size");
    if (p->desc.report_mask != 0 && !partial) return fail(HS_ERR_ARG, "report_mask set but partial is NULL");
    hipStream_t st = (hipStream_t)stream;
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
    const bool plain = p->desc.kernel == HS_KERNEL_PLAIN || (p->desc.kernel == HS_KERNEL_AUTO && a.partial);
    if (plain || a.partial) {
        dim3 grid((unsigned)((n_bins + hs::kBlock - 1) / hs::kBlock), 1);
        hipError_t e = hs::launch_sum_1d(a, p->hmax, p->desc.mode == HS_GREEDY, p->desc.dtype == HS_F16, grid, st);
        if (e != hipSuccess) return fail_hip(e, "harmonic-sum kernel");
    } else {
        s = run_persistent(p, a, 1, st);
        if (s != HS_OK) return s;
    }
    return mark(p, 2, st);
}

hs_status hs_sum_batched(hs_plan *p, const void *x, const int64_t *offsets, int32_t n_spectra, const double *norm,
                         float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand, int64_t cand_capacity,
                         unsigned long long *cand_count, void *stream) {
    if (!p || !x || !offsets) return fail(HS_ERR_ARG, "null argument");
    if (n_spectra < 1 || n_spectra > p->max_groups) return fail(HS_ERR_ARG, "n_spectra out of range");
    if (!aligned_elem(x, p->desc.dtype)) return fail(HS_ERR_ARG, "x must be aligned to its element size");
    if (!snr && !cand) return fail(HS_ERR_ARG, "neither dense outputs nor candidates requested");
    if (snr && !harm) return fail(HS_ERR_ARG, "snr given without harm");
    if (cand && (!cand_count || cand_capacity < 0)) return fail(HS_ERR_ARG, "candidate buffer needs a counter");
    hipStream_t st = (hipStream_t)stream;
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
    if (p->desc.kernel == HS_KERNEL_PLAIN) {
        dim3 grid(hs::kTileBlocksBatched, (unsigned)n_spectra);
        e = hs::launch_sum_1d(a, p->hmax, p->desc.mode == HS_GREEDY, p->desc.dtype == HS_F16, grid, st);
        if (e != hipSuccess) return fail_hip(e, "harmonic-sum kernel");
    } else {
        s = run_persistent(p, a, n_spectra, st);
        if (s != HS_OK) return s;
    }
    return mark(p, 2, st);
}

hs_status hs_sum_2d(hs_plan *p, const void *plane, int64_t n_r, int64_t row_stride, int32_t z_min, int32_t z_max,
                    const double *norm, float *snr, uint8_t *harm, uint8_t *drift, hs_candidate *cand,
                    int64_t cand_capacity, unsigned long long *cand_count, void *stream) {
    if (!p || !plane) return fail(HS_ERR_ARG, "null argument");
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
    // rows == 1 is the 1D layout; keep the plane description for one row too
    if (n_z == 1) {
        sa.rows = 1;
        sa.n_bins = n_r;
    }
    hs_status s = run_norm(p, sa, 1, st);
    if (s != HS_OK) return s;
    hs::Sum2dArgs a{};
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
    e = hs::launch_sum_2d(a, p->hmax, p->desc.mode == HS_GREEDY, p->desc.dtype == HS_F16, st);
    if (e != hipSuccess) return fail_hip(e, "harmonic-sum kernel");
    return mark(p, 2, st);
}

hs_status hs_get_norm(hs_plan *p, int32_t n, double *mu_sigma, float *tables, int32_t *valid, void *stream) {
    if (!p) return fail(HS_ERR_ARG, "null plan");
    if (n < 1 || n > p->last_groups) return fail(HS_ERR_ARG, "n exceeds the groups of the last call");
    if (!mu_sigma && !tables && !valid) return fail(HS_ERR_ARG, "nothing to export");
    hipError_t e = hs::launch_export_norm(p->norm, n, p->desc.harmonics, mu_sigma, tables, valid,
                                          (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "export kernel");
    return HS_OK;
}

hs_status hs_quantize_f16(const float *x, int64_t n, float scale, uint16_t *out, void *stream) {
    if (!x || !out) return fail(HS_ERR_ARG, "null argument");
    if (n < 0) return fail(HS_ERR_ARG, "n < 0");
    if (!(scale > 0.0f) || !(scale < __builtin_inff())) return fail(HS_ERR_ARG, "scale must be positive and finite");
    if (n == 0) return HS_OK;
    hipError_t e = hs::launch_quantize_f16(x, n, scale, out, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "quantise kernel");
    return HS_OK;
}

hs_status hs_plan_set_timing(hs_plan *p, int32_t enable) {
    if (!p) return fail(HS_ERR_ARG, "null plan");
    p->timing = enable != 0;
    p->ev_used = 0;
    return HS_OK;
}

hs_status hs_plan_get_timing(hs_plan *p, int32_t *calls, double *norm_ms, double *sum_ms) {
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
}

const char *hs_status_string(hs_status s) {
    switch (s) {
        case HS_OK: return "ok";
        case HS_ERR_ARG: return "invalid argument";
        case HS_ERR_UNSUPPORTED: return "unsupported";
        case HS_ERR_HIP: return "HIP runtime error";
        case HS_ERR_NOMEM: return "out of memory";
    }
    return "unknown status";
}

const char *hs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
