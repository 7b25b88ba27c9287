/*
 * hs.h -- incoherent harmonic sum on MI355X (gfx950): the C ABI.
 *
 * The operation (Adamek, Roy & Armour, "A Novel Greedy Approach To Harmonic
 * Summing Using GPUs", arXiv:2202.12817):
 *
 *   For every fundamental bin n of a power spectrum x, form the partial sums
 *   S_k of k harmonic elements, k = 1..H, normalise each to an SNR with the
 *   mean and standard deviation of a k-element sum, and keep the best SNR,
 *   its harmonic count and the drift of its last bin (Sec. 2, Eq. (1)-(2)).
 *   Element k is
 *     - simple sum (HS_STANDARD, Sec. 3.1, Eq. (3)):  x[k n];
 *     - greedy sum (HS_GREEDY, Sec. 3.3, Eq. (5), Algorithm 2): the larger of
 *       x[k n + d] and x[k n + d + 1]; when the second is strictly larger the
 *       drift d grows by one.  Step k = 1 compares x[n] and x[n + 1].
 *
 *   The PRESTO-style comparators (Sec. 3.2, Eq. (4), Algorithm 1) index the
 *   output by the LAST bin n of a series instead: stage K (harmonic order K)
 *   sums the bins nearest to h n / K (halves rounded up), in increasing h,
 *   and forms one SNR from its m-element sum:
 *     - HS_PRESTO:      K = 2, 4, 8, ... <= H; h = 1 and the even h <= K
 *                       (m = 1 + K/2);
 *     - HS_PRESTO_ALL:  the same K; every h = 1..K (m = K);
 *     - HS_PRESTO_PLUS: every K = 1..H; every h = 1..K (m = K).
 *   A stage is formed only if its fundamental (the bin nearest to n / K) is
 *   >= first_bin.  harm = the order K of the best stage (its fundamental is
 *   the bin nearest to n / harm), drift = 0, harmonic_mask bit K-1 selects
 *   stage K, fundamental_end bounds the last bin.  These modes run one kernel
 *   (kernel AUTO or PLAIN), support hs_sum_1d without report_mask and
 *   hs_sum_batched with H <= 32, and return HS_ERR_UNSUPPORTED from
 *   hs_sum_2d, the launch shape calls and the tuner.
 *
 * Conventions shared by every entry point:
 *
 *   - Normalisation (reading of Eq. (2) and GetMeanStdev of Algorithms 1-2):
 *     mu1, var1 = population mean and variance of the stored powers of bins
 *     [first_bin, N) (of the whole plane in 2D), each the exact value rounded
 *     once to double; sigma1 = sqrt(var1) rounded once; mu_k = k mu1,
 *     sigma_k = sqrt(k) sigma1.  The float SNR of a k-element sum is
 *     fmaf(S_k, rs_k, nm_k) with rs_k = (float)(1/sigma_k) and
 *     nm_k = (float)(-(mu_k/sigma_k)); S_k is summed in float in harmonic
 *     order.  A caller may supply (mu1, sigma1) instead (`norm` arguments),
 *     or, with hs_plan_desc.norm_kind = HS_NORM_TABLE, the whole per-k table
 *     (mu_k, sigma_k for k = 1..H; Eq. (2) normalises the k-element sum by
 *     the mean and deviation of a k-element sum, which a caller may have
 *     calibrated on its own null): then rs_k = (float)(1/sigma_k) and
 *     nm_k = (float)(-(mu_k/sigma_k)).  sigma1 (any sigma_k of a table) zero
 *     or not finite, or a mean not finite: every output of that spectrum is
 *     zero.
 *   - Truncation: harmonic k of fundamental n is summed only while every bin it
 *     may read is inside the spectrum: k n <= N-1 (simple), k (n+1) <= N-1
 *     (greedy).  Bins below first_bin or at/after fundamental_end are no
 *     fundamental.  Every bin gets an output (zeros where no sum is formed).
 *   - Best partial sum: the largest SNR among the k selected by harmonic_mask,
 *     ties to the smaller k.  Outputs per bin: snr (float), harm = harmonic
 *     count of the best sum (1..H, 0 = none), drift = the drift after that
 *     harmonic (the last summed bin is harm * n + drift; 0 for HS_STANDARD).
 *   - Memory: every array argument is DEVICE memory owned by the caller
 *     (inputs, outputs, candidate buffers, counters), naturally aligned.  The
 *     library owns only the plan and its internal workspace.  Inputs must stay
 *     valid and outputs untouched until the stream has reached the end of the
 *     call.  Powers must be finite.
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream) of the
 *     plan's device, which must be the current device (else HS_ERR_ARG).
 *     Every call only enqueues work; it does not synchronise.
 *   - Errors: argument checks happen before anything is enqueued and return
 *     HS_ERR_ARG / HS_ERR_UNSUPPORTED with nothing launched.  A failing HIP
 *     call returns HS_ERR_HIP.  hs_last_error() returns a message for the
 *     calling thread's last failure.  A plan must not be used from two host
 *     threads at once; calls that overlap on the GPU through one plan race on
 *     its workspace, so enqueue them on one stream.
 */
#ifndef HS_H
#define HS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hs_status {
    HS_OK = 0,
    HS_ERR_ARG = 1,          /* invalid argument (null pointer, size or range) */
    HS_ERR_UNSUPPORTED = 2,  /* valid but not supported by this build (e.g. H > 64) */
    HS_ERR_HIP = 3,          /* a HIP runtime call failed */
    HS_ERR_NOMEM = 4,        /* an allocation failed (the plan's device workspace, or host memory) */
    HS_ERR_INTERNAL = 5      /* unexpected failure inside the library (no exception crosses the ABI) */
} hs_status;

enum { HS_STANDARD = 0, HS_GREEDY = 1,          /* hs_plan_desc.mode */
       HS_PRESTO = 2, HS_PRESTO_ALL = 3, HS_PRESTO_PLUS = 4 };
enum { HS_F32 = 0, HS_F16 = 1 };           /* hs_plan_desc.dtype: stored power type */
/* hs_plan_desc.kernel: which kernel runs.  PLAIN is the design the paper
 * describes for its GPU sum (Sec. 3.1.1): one thread per fundamental bin, a
 * grid per spectrum (per plane row in 2D).  PERSISTENT is, for spectra, the
 * XCD-aware work-queue kernel and, in 2D, the ray-tiled kernel that stages
 * each tile's window of the plane in LDS (used when a tile of ratio width 1
 * fits its budget, about 100 rows on each side of z = 0; wider planes run
 * PLAIN).  AUTO = PERSISTENT for hs_sum_batched (unless the tuner picked
 * PLAIN for the plan) and PLAIN for hs_sum_1d and hs_sum_2d (measured faster
 * there).  hs_sum_1d with report_mask always runs PLAIN.  All give the same
 * results, bit for bit. */
enum { HS_KERNEL_AUTO = 0, HS_KERNEL_PERSISTENT = 1, HS_KERNEL_PLAIN = 2 };
/* hs_plan_desc.norm_kind: what the `norm` argument of the sum calls holds
 * when it is not NULL.  MU_SIGMA: [2] doubles (mu1, sigma1) per spectrum
 * (plane); the k-element sum uses mu_k = k mu1, sigma_k = sqrt(k) sigma1.
 * TABLE: [2][H] doubles per spectrum (plane): mu_1..mu_H, then
 * sigma_1..sigma_H, used as given; norm must then not be NULL. */
enum { HS_NORM_MU_SIGMA = 0, HS_NORM_TABLE = 1 };

#define HS_MAX_HARMONICS 64

/* Plan parameters.  Fill with hs_plan_desc_init, then override. */
typedef struct hs_plan_desc {
    int32_t  harmonics;        /* H, 1..HS_MAX_HARMONICS (default 32; PRESTO modes: 1..32) */
    int32_t  mode;             /* HS_STANDARD, HS_GREEDY (default) or a PRESTO mode */
    int32_t  dtype;            /* HS_F32 or HS_F16 (IEEE binary16 storage, decoded exactly) */
    int32_t  first_bin;        /* >= 1; lowest fundamental and lowest bin in the statistics (default 1) */
    uint64_t harmonic_mask;    /* bit k-1 set: the k-harmonic sum competes for the best; 0 = all (default) */
    uint64_t report_mask;      /* hs_sum_1d only: bit k-1 set: export S_k (default 0) */
    int64_t  fundamental_end;  /* fundamentals >= this give zeros; 0 = no limit (default) */
    int32_t  max_spectra;      /* hs_sum_batched: most spectra per call (default 1024) */
    float    threshold;        /* candidates: snr > threshold (default 6) */
    int32_t  kernel;           /* HS_KERNEL_AUTO (default), HS_KERNEL_PERSISTENT or HS_KERNEL_PLAIN */
    int32_t  norm_kind;        /* HS_NORM_MU_SIGMA (default) or HS_NORM_TABLE: layout of `norm` */
} hs_plan_desc;

/* One candidate: a bin whose best SNR is strictly above the threshold. */
typedef struct hs_candidate {
    uint32_t spectrum;   /* index of the spectrum (0 for hs_sum_2d) */
    uint32_t bin;        /* fundamental bin n (PRESTO modes: last bin; hs_sum_2d: row * n_r + column) */
    float    snr;        /* best SNR */
    uint16_t harm;       /* harmonic count of the best partial sum */
    uint16_t drift;      /* drift after that harmonic */
} hs_candidate;

typedef struct hs_plan hs_plan;

/* Fill *desc with the defaults listed above. */
void hs_plan_desc_init(hs_plan_desc *desc);

/*
 * Validate *desc and create a plan on the current HIP device, allocating its
 * device workspace (one hipMalloc of hs_plan_workspace_bytes: statistics and
 * tables for max_spectra spectra).  *plan is set on success and must be
 * released with hs_plan_destroy.
 */
hs_status hs_plan_create(const hs_plan_desc *desc, hs_plan **plan);

/*
 * Device workspace of a plan with this descriptor, in bytes (host-only
 * arithmetic; validates *desc like hs_plan_create).  It grows with
 * max_spectra: statistics partials, normalisation records and work-queue
 * counters of every spectrum of a call.
 */
hs_status hs_plan_workspace_bytes(const hs_plan_desc *desc, size_t *bytes);

/*
 * Like hs_plan_create, but the plan keeps its device workspace in the
 * caller's buffer: workspace is device memory on the current device, 256-byte
 * aligned, at least hs_plan_workspace_bytes bytes, owned by the caller and
 * kept alive (and not used for anything else) until hs_plan_destroy.  The
 * plan then allocates no device memory.  HS_ERR_ARG for a NULL, misaligned or
 * too small buffer.
 */
hs_status hs_plan_create_in(const hs_plan_desc *desc, void *workspace, size_t bytes, hs_plan **plan);

/* Release the plan (waits for nothing: the caller ensures no call is in flight). */
hs_status hs_plan_destroy(hs_plan *plan);

/*
 * One spectrum (Eq. (3) or Algorithm 2 over all of its bins).
 *   x        [n_bins] powers, dtype of the plan.  2 <= n_bins < 2^30.
 *   norm     NULL: statistics from x; else [2] doubles (mu1, sigma1), or
 *            [2][H] doubles (mu_k, then sigma_k) with HS_NORM_TABLE.
 *   snr      [n_bins] float, harm [n_bins] uint8, drift [n_bins] uint8: dense
 *            outputs indexed by fundamental bin; drift may be NULL.
 *   partial  NULL, or [popcount(report_mask)][n_bins] floats: S_k for each
 *            reported k in increasing k (0 where fewer than k harmonics fit).
 */
hs_status hs_sum_1d(hs_plan *plan, const void *x, int64_t n_bins, const double *norm,
                    float *snr, uint8_t *harm, uint8_t *drift, float *partial, void *stream);

/*
 * A batch of independent spectra of any lengths, each with its own statistics,
 * in one launch sequence (Sec. 4.3 processes 1024 spectra at once).
 *   x          concatenated powers; spectrum s is x[offsets[s] .. offsets[s+1]).
 *   offsets    [n_spectra + 1] int64, non-decreasing, offsets[0] = 0; each
 *              spectrum 2 <= length < 2^30.  (Lengths are read on the device
 *              and not re-validated there: keep them within these bounds.)
 *   n_spectra  1..max_spectra of the plan (max_spectra <= 65535).
 *   norm       NULL or [n_spectra][2] doubles (mu1, sigma1 per spectrum), or
 *              [n_spectra][2][H] doubles with HS_NORM_TABLE.
 *   snr/harm/drift  NULL, or dense outputs indexed like x.
 *   cand       NULL, or [cand_capacity] records of every bin with snr >
 *              threshold, in unspecified order; *cand_count (device, zeroed
 *              by the call) receives the true number of such bins even when
 *              it exceeds cand_capacity (then only cand_capacity are written).
 *   At least one of snr or cand must be given.
 */
hs_status hs_sum_batched(hs_plan *plan, const void *x, const int64_t *offsets, int32_t n_spectra,
                         const double *norm, float *snr, uint8_t *harm, uint8_t *drift,
                         hs_candidate *cand, int64_t cand_capacity,
                         unsigned long long *cand_count, void *stream);

/*
 * The f-fdot form (Sec. 1 names it; reading: harmonic k of fundamental (r, z)
 * is at column k r and row k z, and the sum stops before the first row outside
 * [z_min, z_max]; greedy drift moves along r only; statistics over the plane).
 *   plane      row i (z = z_min + i) starts at plane + i * row_stride; n_r
 *              columns.  row_stride >= n_r.  2 <= n_r < 2^30.
 *   z_min <= 0 <= z_max is not required; rows are z_min..z_max.
 *   norm       NULL or [2] doubles (mu1, sigma1), or [2][H] with HS_NORM_TABLE.
 *   snr/harm/drift  NULL, or dense [n_z][n_r] outputs (row stride n_r).
 *   cand/cand_capacity/cand_count  as for hs_sum_batched (bin = i * n_r + r).
 */
hs_status hs_sum_2d(hs_plan *plan, const void *plane, int64_t n_r, int64_t row_stride,
                    int32_t z_min, int32_t z_max, const double *norm,
                    float *snr, uint8_t *harm, uint8_t *drift,
                    hs_candidate *cand, int64_t cand_capacity,
                    unsigned long long *cand_count, void *stream);

/*
 * Equal-length spectra in the interleaved layout of Sec. 3.1.1 (the same bin
 * of different spectra side by side): bin m of spectrum s at
 * x[m * n_spectra + s].  Each spectrum (column) gets its own statistics and
 * the sums of the plan's mode (HS_STANDARD or HS_GREEDY; others return
 * HS_ERR_UNSUPPORTED), bit for bit those of hs_sum_batched on the same
 * spectra stored one after another.  The plan's kernel choice is ignored.
 *   x          [n_bins][n_spectra] powers, dtype of the plan; n_bins >= 2,
 *              n_bins * n_spectra < 2^30, 1 <= n_spectra <= max_spectra.
 *   norm       NULL or [n_spectra][2] doubles (mu1, sigma1 per spectrum), or
 *              [n_spectra][2][H] with HS_NORM_TABLE.
 *   snr/harm/drift  NULL, or dense [n_bins][n_spectra] outputs (interleaved
 *              like x); drift may be NULL.
 *   cand/cand_capacity/cand_count  as for hs_sum_batched (spectrum = s,
 *              bin = m).  At least one of snr or cand must be given.
 */
hs_status hs_sum_interleaved(hs_plan *plan, const void *x, int64_t n_bins, int32_t n_spectra,
                             const double *norm, float *snr, uint8_t *harm, uint8_t *drift,
                             hs_candidate *cand, int64_t cand_capacity,
                             unsigned long long *cand_count, void *stream);

/*
 * The transpose into the interleaved layout (the preprocessing that
 * Sec. 3.1.1 says the layout costs): out[m * n_spectra + s] = x[s * n_bins + m]
 * for n_spectra spectra of n_bins elements of elem_bytes (2 or 4) bytes.
 * Device buffers of n_bins * n_spectra elements that must not overlap;
 * stream-ordered like the sum calls.  No plan needed.
 */
hs_status hs_interleave(const void *x, int64_t n_bins, int32_t n_spectra, int32_t elem_bytes,
                        void *out, void *stream);

/*
 * The power spectrum the sum runs on, from complex FFT bins (the step before
 * the harmonic sum; Sec. 2 names power-spectrum calculation with
 * inter-binning).  fft: n_bins complex values (float re, float im pairs,
 * 8-byte aligned).  interbin 0: out[m] = fl(fl(fl(re*re) + fl(im*im)) * scale),
 * n_bins floats.  interbin 1: 2 n_bins - 1 floats, out[2m] = bin m as above
 * and out[2m+1] = the half bin between m and m + 1, whose amplitude is
 * estimated as (pi/4)(F_m - F_{m+1}):  fl(fl(fl(dr*dr) + fl(di*di)) * s_h)
 * with dr, di the float differences and s_h = fl32(scale * fl32(pi^2/16)).
 * scale > 0 (e.g. 1 / (N sigma^2) for unit mean noise power); 1 <= n_bins < 2^31;
 * fft and out must not overlap.  Stream-ordered; no plan needed.
 */
hs_status hs_power_spectrum(const void *fft, int64_t n_bins, int32_t interbin, float scale, float *out,
                            void *stream);

/*
 * Peak clustering of dense outputs (the step after the sum): a candidate
 * (snr > threshold, strict float compare, harm > 0) is kept if no bin of the
 * same spectrum within radius bins beats it -- a larger snr, or an equal snr
 * at a lower bin -- so kept peaks are more than radius bins apart.
 *   snr, harm, drift   dense outputs of a sum call (drift may be NULL: 0);
 *   offsets            NULL: one spectrum of n_bins (n_spectra = 1); else
 *                      [n_spectra + 1] device offsets as for hs_sum_batched
 *                      (n_bins = total bins, 1 <= n_spectra <= 65535);
 *   cand/cand_capacity/cand_count   as for hs_sum_batched (bin = bin within
 *                      its spectrum; *cand_count zeroed by the call).
 * radius >= 0 (0: every candidate).  Stream-ordered; no plan needed.
 */
hs_status hs_cluster_peaks(const float *snr, const uint8_t *harm, const uint8_t *drift, const int64_t *offsets,
                           int64_t n_bins, int32_t n_spectra, int32_t radius, float threshold,
                           hs_candidate *cand, int64_t cand_capacity, unsigned long long *cand_count,
                           void *stream);

/*
 * hs_sum_batched without a plan, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same launch sequence and kernels as hs_sum_batched with a plan made
 * from *desc (persistent kernel, default launch shape; the same results bit
 * for bit), with its workspace in a static device array of the library
 * (4 MiB per device, held until the process ends) instead of plan memory.
 * Nothing is allocated, on the host or the device.  Arguments as for
 * hs_sum_batched; desc->max_spectra is ignored and n_spectra must be
 * 1..1024 (HS_ERR_ARG beyond).  Every call on one device shares that array:
 * each call clears what must start at zero, and calls that overlap on one GPU
 * (different streams, or host threads) race on it -- enqueue them on one
 * stream.  hs_get_norm does not apply (no plan).
 */
hs_status hs_sum_batched_static(const hs_plan_desc *desc, const void *x, const int64_t *offsets, int32_t n_spectra,
                                const double *norm, float *snr, uint8_t *harm, uint8_t *drift,
                                hs_candidate *cand, int64_t cand_capacity,
                                unsigned long long *cand_count, void *stream);

/*
 * Export the normalisation used by the most recent sum call on this plan
 * (stream-ordered device-to-device copy of its first n entries).
 *   mu_sigma  [2 n] doubles (mu1, sigma1; with HS_NORM_TABLE mu_1 and
 *             sigma_1 of the caller's table); tables NULL or [n][2][H] floats
 *             (rs_k for k = 1..H, then nm_k for k = 1..H); valid NULL or [n]
 *             int32 (1 = usable normalisation, 0 = degenerate: zero outputs).
 */
hs_status hs_get_norm(hs_plan *plan, int32_t n, double *mu_sigma, float *tables,
                      int32_t *valid, void *stream);

/*
 * FP16 storage of powers: out[i] = fp16_rne(clamp((float)x[i] / scale, +-65504))
 * (one correctly rounded float division, then round-to-nearest-even to
 * binary16).  scale > 0 and finite.  out is binary16 bit patterns.
 */
hs_status hs_quantize_f16(const float *x, int64_t n, float scale, uint16_t *out, void *stream);

/*
 * Stage timing (profiling aid).  With timing enabled, every sum call records
 * HIP events on its stream before and after its normalisation stage and after
 * its harmonic-sum kernel.  hs_plan_get_timing waits for the recorded events,
 * returns the number of timed calls and the summed milliseconds of the two
 * stages (any pointer may be NULL), and clears the record.
 */
hs_status hs_plan_set_timing(hs_plan *plan, int32_t enable);
hs_status hs_plan_get_timing(hs_plan *plan, int32_t *calls, double *norm_ms, double *sum_ms);

/*
 * Graph capture.  Every sum entry point enqueues kernels only (no memset, no
 * copy, no allocation, no synchronisation), so a caller may record it into
 * its own graph with stream capture; each replay then reuses the plan's
 * workspace, so replays through one plan must not overlap on the GPU.  Stage
 * timing must be off while the caller's stream captures (HS_ERR_ARG).
 *
 * hs_plan_set_graph(plan, 1) makes the library do this itself: the first
 * call with a given argument set (entry point, every pointer and size) is
 * recorded into a hipGraph and every later call with the same arguments
 * replays it with one graph launch on the caller's stream (the same results:
 * the graph holds the same kernels).  The 8 most recently used argument sets
 * are kept; dropping one waits for its last replay.  Timed calls and calls on
 * a capturing stream run without the cache.  Disabling (0) waits for the last
 * replay of every cached graph and releases them.  hs_plan_graph_info returns
 * the number of recorded graphs and of replays since the plan was created.
 */
hs_status hs_plan_set_graph(hs_plan *plan, int32_t enable);
hs_status hs_plan_graph_info(hs_plan *plan, int64_t *captures, int64_t *replays);

/*
 * Launch shape of the persistent kernel (hs_sum_batched and the persistent
 * hs_sum_1d): fundamentals per lane (1, 2 or 4) and resident workgroups of
 * 256 threads per CU (1..8, bounded by the kernel's occupancy: 6 or 7 on
 * gfx950); for a plan with
 * HS_KERNEL_AUTO, fundamentals_per_lane 0 makes hs_sum_batched run the plain
 * kernel (workgroups_per_cu ignored; hs_plan_get_launch reports 0, 0).  The
 * results do not depend on the shape.  Default: 2 and 4 for FP32, 4 and 5
 * for FP16 (environment HS_XCD_F and HS_XCD_WGS_PER_CU override the
 * defaults at plan creation).
 * Setting a new shape drops the plan's cached graphs.
 */
hs_status hs_plan_set_launch(hs_plan *plan, int32_t fundamentals_per_lane, int32_t workgroups_per_cu);
hs_status hs_plan_get_launch(hs_plan *plan, int32_t *fundamentals_per_lane, int32_t *workgroups_per_cu);

/*
 * Autotuner of the launch shape for a batch (arguments as hs_sum_batched; the
 * work of Sec. 4.3 is batches of many spectra, whose best shape depends on
 * the device and on the batch).  Runs hs_sum_batched once with the current
 * shape, then, unless cache_path names a file with an entry for this key,
 * times every shape (one warm-up and the median of three calls each), keeps
 * the fastest on the plan and appends a line to cache_path (if not NULL).
 * The key is: device architecture, CU and XCD counts, harmonic bucket, mode,
 * dtype, output kind, and the powers of two below the total bins and the
 * number of spectra.  For an HS_KERNEL_AUTO plan the plain kernel is one of
 * the shapes.  On return the outputs hold the result of a complete call.
 * Synchronises the stream (host-blocking); HS_ERR_ARG for a plan with
 * HS_KERNEL_PLAIN, with timing enabled, or on a capturing stream.
 */
hs_status hs_plan_tune_batched(hs_plan *plan, const void *x, const int64_t *offsets, int32_t n_spectra,
                               const double *norm, float *snr, uint8_t *harm, uint8_t *drift,
                               hs_candidate *cand, int64_t cand_capacity,
                               unsigned long long *cand_count, const char *cache_path, void *stream);

const char *hs_status_string(hs_status status);
const char *hs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HS_H */
