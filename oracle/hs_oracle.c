/*
 * CPU oracle of the incoherent harmonic sum -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  The GPU library shares no code with it and never calls
 * it.  Every loop below is the plain, slow, one-fundamental-at-a-time reading
 * of the paper ("A Novel Greedy Approach To Harmonic Summing Using GPUs",
 * Adamek, Roy & Armour, arXiv:2202.12817):
 *
 *   - the simple harmonic sum, Sec. 3.1, Eq. (3): element k of the sum for
 *     fundamental bin n is x[k n];
 *   - the greedy harmonic sum, Sec. 3.3, Eq. (5) and Algorithm 2: element k is
 *     the larger of x[k n + d] and x[k n + d + 1]; when the second one is
 *     strictly larger the drift d grows by one (the fundamental step k = 1
 *     compares x[n] and x[n + 1]);
 *   - the SNR of every partial sum and the running maximum, Sec. 2, Eq. (2),
 *     normalised with the mean and standard deviation of a partial sum of k
 *     elements (tables computed by the Python side of the oracle);
 *   - the PRESTO-style sums the paper compares against, Sec. 3.2, Eq. (4) and
 *     Algorithm 1 (PRESTO, PRESTO_all, PRESTO+), at the end of this file.
 *
 * Two precisions:
 *   f32: the partial sums are accumulated in float in harmonic order and the
 *        SNR of a k-element sum is the single-rounding fused value
 *        fmaf(S_k, rs[k-1], nm[k-1]), with rs = 1/sigma_k and nm = -mu_k/sigma_k
 *        rounded once to float.  This mirrors the precision in which the GPU
 *        takes the argmax decision, so chosen harmonic counts and drifts can be
 *        compared bit for bit.
 *   f64: sums in double, SNR = (S_k - mu_k) / sigma_k in double.  This is the
 *        accuracy reference for the float SNR values.
 *
 * Truncation (a reading; the paper loops over all H harmonics of every bin):
 * harmonic k of fundamental n is summed only while every bin it may read lies
 * inside the array: k n <= len - 1 (simple) or k (n + 1) <= len - 1 (greedy,
 * whose drift before step k is at most k - 1).  Fundamentals with no harmonic
 * left produce zeros.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no contraction of the
 * explicit float arithmetic; x86-64 SSE arithmetic has no excess precision).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* Number of harmonics summed for fundamental n of an array of len bins. */
static int64_t keff(int64_t n, int64_t len, int32_t H, int32_t greedy)
{
    if (n < 1) return 0;
    int64_t reach = greedy ? n + 1 : n;
    int64_t k = (len - 1) / reach;
    return k < H ? k : H;
}

/* Bounds-checked read: an out-of-range index is a bug in the oracle itself. */
static inline float rd32(const float *row, int64_t len, int64_t m)
{
    if (m < 0 || m >= len) abort();
    return row[m];
}

/*
 * One fundamental n in float.  rows[k-1] is the array harmonic k reads from
 * (the same array for every k in 1D; row k z of the plane in 2D).  K is the
 * number of harmonics to sum.  Outputs the best SNR, its harmonic count (0 when
 * no partial sum was eligible) and the drift after that harmonic, plus the
 * requested partial sums.
 */
static void one_f32(const float *const *rows, int64_t len, int64_t n, int64_t K,
                    int32_t greedy, uint64_t kmask, const float *rs, const float *nm,
                    float *o_snr, uint8_t *o_harm, uint8_t *o_drift,
                    int32_t n_report, const int32_t *report_k, float *o_partial,
                    int64_t partial_stride)
{
    float S = 0.0f, best = 0.0f;
    int64_t d = 0;
    int32_t kb = 0, db = 0;
    for (int32_t r = 0; r < n_report; ++r) o_partial[r * partial_stride] = 0.0f;
    for (int64_t k = 1; k <= K; ++k) {
        const float *row = rows[k - 1];
        float v;
        if (greedy) {
            float a = rd32(row, len, k * n + d);
            float b = rd32(row, len, k * n + d + 1);
            if (b > a) { d += 1; v = b; } else { v = a; }
        } else {
            v = rd32(row, len, k * n);
        }
        S = S + v;
        float snr = fmaf(S, rs[k - 1], nm[k - 1]);
        for (int32_t r = 0; r < n_report; ++r)
            if (report_k[r] == k) o_partial[r * partial_stride] = S;
        if ((kmask >> (k - 1)) & 1u) {
            if (kb == 0 || snr > best) { best = snr; kb = (int32_t)k; db = (int32_t)d; }
        }
    }
    *o_snr = kb ? best : 0.0f;
    *o_harm = (uint8_t)kb;
    *o_drift = (uint8_t)db;
}

/* The same procedure in double precision. */
static void one_f64(const float *const *rows, int64_t len, int64_t n, int64_t K,
                    int32_t greedy, uint64_t kmask, const double *mu, const double *sig,
                    double *o_snr, uint8_t *o_harm, uint8_t *o_drift,
                    int32_t n_report, const int32_t *report_k, double *o_partial,
                    int64_t partial_stride)
{
    double S = 0.0, best = 0.0;
    int64_t d = 0;
    int32_t kb = 0, db = 0;
    for (int32_t r = 0; r < n_report; ++r) o_partial[r * partial_stride] = 0.0;
    for (int64_t k = 1; k <= K; ++k) {
        const float *row = rows[k - 1];
        double v;
        if (greedy) {
            float a = rd32(row, len, k * n + d);
            float b = rd32(row, len, k * n + d + 1);
            if (b > a) { d += 1; v = b; } else { v = a; }
        } else {
            v = rd32(row, len, k * n);
        }
        S = S + v;
        double snr = (S - mu[k - 1]) / sig[k - 1];
        for (int32_t r = 0; r < n_report; ++r)
            if (report_k[r] == k) o_partial[r * partial_stride] = S;
        if ((kmask >> (k - 1)) & 1u) {
            if (kb == 0 || snr > best) { best = snr; kb = (int32_t)k; db = (int32_t)d; }
        }
    }
    *o_snr = kb ? best : 0.0;
    *o_harm = (uint8_t)kb;
    *o_drift = (uint8_t)db;
}

#define HS_ORACLE_MAX_H 64

/*
 * 1D spectrum x[0..len).  Fundamentals are idx[o] for o < n_out (idx == NULL:
 * every bin, o = n).  Bins below first_bin or at/after n_end are no
 * fundamental and get zeros.  partial: n_report rows of n_out values.
 */
void hso_1d_f32(const float *x, int64_t len, int32_t H, int32_t greedy,
                int64_t first_bin, int64_t n_end, uint64_t kmask,
                const float *rs, const float *nm, const int64_t *idx, int64_t n_out,
                float *snr, uint8_t *harm, uint8_t *drift,
                int32_t n_report, const int32_t *report_k, float *partial)
{
    const float *rows[HS_ORACLE_MAX_H];
    if (H < 1 || H > HS_ORACLE_MAX_H) abort();
    for (int32_t k = 0; k < H; ++k) rows[k] = x;
    for (int64_t o = 0; o < n_out; ++o) {
        int64_t n = idx ? idx[o] : o;
        int64_t K = (n >= first_bin && n < n_end) ? keff(n, len, H, greedy) : 0;
        one_f32(rows, len, n, K, greedy, kmask, rs, nm, snr + o, harm + o, drift + o,
                partial ? n_report : 0, report_k, partial ? partial + o : NULL, n_out);
    }
}

void hso_1d_f64(const float *x, int64_t len, int32_t H, int32_t greedy,
                int64_t first_bin, int64_t n_end, uint64_t kmask,
                const double *mu, const double *sig, const int64_t *idx, int64_t n_out,
                double *snr, uint8_t *harm, uint8_t *drift,
                int32_t n_report, const int32_t *report_k, double *partial)
{
    const float *rows[HS_ORACLE_MAX_H];
    if (H < 1 || H > HS_ORACLE_MAX_H) abort();
    for (int32_t k = 0; k < H; ++k) rows[k] = x;
    for (int64_t o = 0; o < n_out; ++o) {
        int64_t n = idx ? idx[o] : o;
        int64_t K = (n >= first_bin && n < n_end) ? keff(n, len, H, greedy) : 0;
        one_f64(rows, len, n, K, greedy, kmask, mu, sig, snr + o, harm + o, drift + o,
                partial ? n_report : 0, report_k, partial ? partial + o : NULL, n_out);
    }
}

/*
 * Number of harmonics a fundamental in row z of a plane spanning rows
 * z_min..z_max can sum before harmonic k z leaves the plane (a reading: the
 * paper names the f-fdot sum but gives no formula; harmonic k of (r, z) is
 * taken at (k r, k z) and the sum stops at the first row outside the plane).
 */
static int64_t kz_limit(int32_t z, int32_t z_min, int32_t z_max, int32_t H)
{
    if (z == 0) return H;
    int64_t k = z > 0 ? (int64_t)z_max / z : (int64_t)z_min / z;
    return k < H ? k : H;
}

/*
 * 2D f-fdot plane: row i holds z = z_min + i, n_r columns at row stride
 * `stride`.  Fundamentals are flat indices idx[o] = i n_r + r (idx == NULL:
 * all rows, all columns, o = i n_r + r).  Drift moves along r only.
 */
void hso_2d_f32(const float *plane, int64_t n_r, int64_t stride, int32_t z_min, int32_t z_max,
                int32_t H, int32_t greedy, int64_t first_bin, int64_t n_end, uint64_t kmask,
                const float *rs, const float *nm, const int64_t *idx, int64_t n_out,
                float *snr, uint8_t *harm, uint8_t *drift)
{
    const float *rows[HS_ORACLE_MAX_H];
    int64_t n_z = (int64_t)z_max - z_min + 1;
    if (H < 1 || H > HS_ORACLE_MAX_H) abort();
    for (int64_t o = 0; o < n_out; ++o) {
        int64_t flat = idx ? idx[o] : o;
        int64_t i = flat / n_r, r = flat % n_r;
        int32_t z = (int32_t)(z_min + i);
        if (i < 0 || i >= n_z) abort();
        int64_t K = 0;
        if (r >= first_bin && r < n_end) {
            K = keff(r, n_r, H, greedy);
            int64_t kz = kz_limit(z, z_min, z_max, H);
            if (kz < K) K = kz;
        }
        for (int64_t k = 1; k <= K; ++k) {
            int64_t row = k * z - z_min;
            if (row < 0 || row >= n_z) abort();
            rows[k - 1] = plane + row * stride;
        }
        one_f32(rows, n_r, r, K, greedy, kmask, rs, nm, snr + o, harm + o, drift + o,
                0, NULL, NULL, 0);
    }
}

void hso_2d_f64(const float *plane, int64_t n_r, int64_t stride, int32_t z_min, int32_t z_max,
                int32_t H, int32_t greedy, int64_t first_bin, int64_t n_end, uint64_t kmask,
                const double *mu, const double *sig, const int64_t *idx, int64_t n_out,
                double *snr, uint8_t *harm, uint8_t *drift)
{
    const float *rows[HS_ORACLE_MAX_H];
    int64_t n_z = (int64_t)z_max - z_min + 1;
    if (H < 1 || H > HS_ORACLE_MAX_H) abort();
    for (int64_t o = 0; o < n_out; ++o) {
        int64_t flat = idx ? idx[o] : o;
        int64_t i = flat / n_r, r = flat % n_r;
        int32_t z = (int32_t)(z_min + i);
        if (i < 0 || i >= n_z) abort();
        int64_t K = 0;
        if (r >= first_bin && r < n_end) {
            K = keff(r, n_r, H, greedy);
            int64_t kz = kz_limit(z, z_min, z_max, H);
            if (kz < K) K = kz;
        }
        for (int64_t k = 1; k <= K; ++k) {
            int64_t row = k * z - z_min;
            if (row < 0 || row >= n_z) abort();
            rows[k - 1] = plane + row * stride;
        }
        one_f64(rows, n_r, r, K, greedy, kmask, mu, sig, snr + o, harm + o, drift + o,
                0, NULL, NULL, 0);
    }
}

/*
 * PRESTO-style sums (Sec. 3.2, Eq. (4), Algorithm 1), indexed by the LAST bin
 * n of a harmonic series rather than by its fundamental.  Stage K (harmonic
 * order K) sums the bins nearest to h n / K for the harmonics h it includes,
 * in increasing h, and forms one SNR when the stage is complete.  Readings:
 *   - "Round": nearest integer, halves rounded up: floor((2 h n + K) / (2 K));
 *   - variant 2 (PRESTO): stages K = 2, 4, 8, ... <= H, harmonics h = 1 and
 *     the even h <= K (the paper's PRESTO sums only the even harmonics above
 *     the fundamental);
 *     variant 3 (PRESTO_all): the same stages, every harmonic h = 1..K;
 *     variant 4 (PRESTO+): every stage K = 1..H, every harmonic h = 1..K;
 *   - a stage of m summed elements is normalised with the m-element mean and
 *     standard deviation (Eq. (2)), so a PRESTO stage K uses m = 1 + K/2;
 *   - stage K is formed only if its fundamental bin, the lowest bin it reads,
 *     is >= first_bin; the highest bin it reads is n itself;
 *   - the best stage: the largest SNR among the stages selected by kmask
 *     (bit K-1), ties to the smaller K; harm = its K (its fundamental is the
 *     bin nearest to n / K), 0 when no stage was formed.
 */
#define HSO_PRESTO 2
#define HSO_PRESTO_ALL 3
#define HSO_PRESTO_PLUS 4

/* The bin nearest to h n / K, halves rounded up. */
static int64_t nearest_bin(int64_t h, int64_t n, int64_t K)
{
    return (2 * h * n + K) / (2 * K);
}

static int stage_formed(int32_t variant, int64_t K)
{
    if (variant == HSO_PRESTO_PLUS) return 1;
    return K >= 2 && (K & (K - 1)) == 0;     /* powers of two from 2 */
}

static int harmonic_summed(int32_t variant, int64_t h)
{
    return variant != HSO_PRESTO || h == 1 || h % 2 == 0;
}

void hso_presto_f32(const float *x, int64_t len, int32_t H, int32_t variant,
                    int64_t first_bin, int64_t n_end, uint64_t kmask,
                    const float *rs, const float *nm, const int64_t *idx, int64_t n_out,
                    float *snr, uint8_t *harm)
{
    if (H < 1 || H > HS_ORACLE_MAX_H) abort();
    if (variant < HSO_PRESTO || variant > HSO_PRESTO_PLUS) abort();
    for (int64_t o = 0; o < n_out; ++o) {
        int64_t n = idx ? idx[o] : o;
        float best = 0.0f;
        int32_t kb = 0;
        for (int64_t K = 1; K <= H && n >= first_bin && n < n_end; ++K) {
            if (!stage_formed(variant, K) || nearest_bin(1, n, K) < first_bin) continue;
            float S = 0.0f;
            int64_t m = 0;
            for (int64_t h = 1; h <= K; ++h) {
                if (!harmonic_summed(variant, h)) continue;
                S = S + rd32(x, len, nearest_bin(h, n, K));
                m += 1;
            }
            float v = fmaf(S, rs[m - 1], nm[m - 1]);
            if ((kmask >> (K - 1)) & 1u) {
                if (kb == 0 || v > best) { best = v; kb = (int32_t)K; }
            }
        }
        snr[o] = kb ? best : 0.0f;
        harm[o] = (uint8_t)kb;
    }
}

void hso_presto_f64(const float *x, int64_t len, int32_t H, int32_t variant,
                    int64_t first_bin, int64_t n_end, uint64_t kmask,
                    const double *mu, const double *sig, const int64_t *idx, int64_t n_out,
                    double *snr, uint8_t *harm)
{
    if (H < 1 || H > HS_ORACLE_MAX_H) abort();
    if (variant < HSO_PRESTO || variant > HSO_PRESTO_PLUS) abort();
    for (int64_t o = 0; o < n_out; ++o) {
        int64_t n = idx ? idx[o] : o;
        double best = 0.0;
        int32_t kb = 0;
        for (int64_t K = 1; K <= H && n >= first_bin && n < n_end; ++K) {
            if (!stage_formed(variant, K) || nearest_bin(1, n, K) < first_bin) continue;
            double S = 0.0;
            int64_t m = 0;
            for (int64_t h = 1; h <= K; ++h) {
                if (!harmonic_summed(variant, h)) continue;
                S = S + rd32(x, len, nearest_bin(h, n, K));
                m += 1;
            }
            double v = (S - mu[m - 1]) / sig[m - 1];
            if ((kmask >> (K - 1)) & 1u) {
                if (kb == 0 || v > best) { best = v; kb = (int32_t)K; }
            }
        }
        snr[o] = kb ? best : 0.0;
        harm[o] = (uint8_t)kb;
    }
}
