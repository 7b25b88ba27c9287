/*
 * l2_model.c -- a CPU model of one XCD's L2 under the harmonic walk's access
 * stream, used to compare schedules of the batched greedy sum (and of the
 * f-fdot plane) before spending GPU time on them.  Not part of the library
 * or the tests; numbers from it are design estimates, stated beside the
 * measured counters.
 *
 * The cache: 4 MiB, 128-byte lines, 16 ways, LRU, set index from a hash of
 * the line address.  A wave of 64 fundamentals at harmonic k touches the
 * lines of its 64 greedy pairs (one request per distinct line per wave
 * instruction); drifts follow a fair coin per step.
 *
 *   cc -O2 -o l2_model l2_model.c
 *   python -c "import synthetic; print(*synthetic.config3_lengths()[:8])" | ./l2_model chunks F W [desc]
 *   ... | ./l2_model front R
 *   ./l2_model plane n_r U H W f_lo f_hi
 *
 * chunks: the persistent kernel's schedule -- spectra cut into chunks of
 *   256 F fundamentals (doubling per class as the harmonic count halves),
 *   32 CUs x W workgroups of 4 waves walking adjacent chunks in order
 *   (desc: chunks of each spectrum in decreasing n), the waves interleaved
 *   one harmonic step at a time.
 * front: the same work in the order of the position k n: passes over R
 *   resident fundamentals, every (wave, harmonic) event of a pass executed in
 *   increasing position (the ideal of a front-paced schedule).
 * plane: the f-fdot plane (H harmonics, rows |z| <= U) walked in ray families
 *   f_lo..f_hi (64 ratio units, 64-column items), W workgroups of 4 waves.
 * Output: L2 requests, misses, hit rate and the bytes fetched beyond the L2
 * per bin (per plane element).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { WAYS = 16, SETS = 2048 };   /* 4 MiB of 128-byte lines */
static uint64_t tag[SETS * WAYS], stamp[SETS * WAYS], clk, req, miss;
static uint32_t rng_state = 12345u;

static int coin(void) {
    rng_state = rng_state * 1664525u + 1013904223u;
    return (rng_state >> 16) & 1;
}

static void touch(uint64_t line) {
    const uint64_t h = line ^ (line >> 11) ^ (line >> 22) ^ (line >> 33);
    uint64_t *t = tag + (h & (SETS - 1)) * WAYS, *s = stamp + (h & (SETS - 1)) * WAYS;
    int lru = 0;
    ++req;
    ++clk;
    for (int w = 0; w < WAYS; ++w) {
        if (t[w] == line + 1) {
            s[w] = clk;
            return;
        }
        if (s[w] < s[lru]) lru = w;
    }
    ++miss;
    t[lru] = line + 1;
    s[lru] = clk;
}

static const int H = 32;
static int keff(int64_t n, int64_t len) {
    if (n < 1 || n >= len) return 0;
    const int64_t k = (len - 1) / (n + 1);
    return k < H ? (int)k : H;
}

/* the lines of one wave's greedy pairs at harmonic k (fundamentals n0..n0+63 of a spectrum at off) */
static void wave_step(int64_t off, int64_t len, int64_t n0, int64_t n_hi, int k, uint8_t *d) {
    uint64_t last = ~0ull;
    for (int l = 0; l < 64; ++l) {
        const int64_t n = n0 + l;
        if (n >= n_hi || k > keff(n, len)) continue;
        const int64_t p = off + k * n + d[l];
        const uint64_t l0 = (uint64_t)(p * 4) >> 7, l1 = (uint64_t)((p + 1) * 4 + 3) >> 7;
        if (l0 != last) touch(l0);
        if (l1 != l0) touch(l1);
        last = l1;
        d[l] += coin();
    }
}

static int read_lengths(int64_t *lens, int cap) {
    int n = 0;
    while (n < cap && scanf("%ld", &lens[n]) == 1) ++n;
    return n;
}

typedef struct { int64_t off, len, lo, hi; } Chunk;
typedef struct { Chunk c; int64_t p0; int k, active; uint8_t d[16][64]; } Cursor;

static void model_chunks(int F, int wpc, int desc) {
    static int64_t lens[100000];
    const int ns = read_lengths(lens, 100000);
    const int CH = 256 * F;
    size_t nc = 0, cap = 1 << 22;
    Chunk *cl = malloc(cap * sizeof(Chunk));
    int64_t off = 0;
    for (int s = 0; s < ns; ++s) {
        const int64_t len = lens[s];
        int64_t b[7];
        b[0] = 0;
        for (int j = 1; j <= 6; ++j) {
            int64_t v = j == 6 ? len : (len - 1) / ((H >> j) + 1);
            if (v < b[j - 1]) v = b[j - 1];
            b[j] = v > len ? len : v;
        }
        const size_t first = nc;
        for (int j = 0; j < 6; ++j)
            for (int64_t lo = b[j]; lo < b[j + 1]; lo += (int64_t)CH << j)
                cl[nc++] = (Chunk){off, len, lo, lo + ((int64_t)CH << j) < b[j + 1] ? lo + ((int64_t)CH << j) : b[j + 1]};
        if (desc)
            for (size_t i = 0; i < (nc - first) / 2; ++i) {
                Chunk t = cl[first + i];
                cl[first + i] = cl[nc - 1 - i];
                cl[nc - 1 - i] = t;
            }
        off += len;
    }
    const int R = 32 * wpc;
    Cursor *cu = calloc(R, sizeof(Cursor));
    size_t next = 0;
    int live = 0;
    for (int r = 0; r < R && next < nc; ++r) {
        cu[r].c = cl[next++];
        cu[r].p0 = cu[r].c.lo;
        cu[r].k = 1;
        cu[r].active = 1;
        ++live;
    }
    while (live) {
        for (int r = 0; r < R; ++r) {
            Cursor *u = &cu[r];
            if (!u->active) continue;
            const int KW = keff(u->p0 < 1 ? 1 : u->p0, u->c.len);
            if (u->k <= KW) {
                for (int f = 0; f < F; ++f)
                    for (int w = 0; w < 4; ++w)
                        wave_step(u->c.off, u->c.len, u->p0 + f * 256 + w * 64, u->c.hi, u->k, u->d[f * 4 + w]);
                u->k++;
            }
            if (u->k > KW) {
                u->p0 += CH;
                u->k = 1;
                memset(u->d, 0, sizeof u->d);
                if (u->p0 >= u->c.hi) {
                    if (next < nc) {
                        u->c = cl[next++];
                        u->p0 = u->c.lo;
                    } else {
                        u->active = 0;
                        --live;
                    }
                }
            }
        }
    }
    printf("chunks F=%d W=%d%s: %d spectra, requests %llu misses %llu hit %.1f%% fetched %.2f B/bin\n", F, wpc,
           desc ? " descending" : "", ns, (unsigned long long)req, (unsigned long long)miss,
           100.0 * (double)(req - miss) / (double)req, 128.0 * (double)miss / (double)off);
}

typedef struct { uint64_t pos; uint32_t wave; uint16_t k; } Event;
static int by_pos(const void *a, const void *b) {
    const Event *x = a, *y = b;
    return x->pos < y->pos ? -1 : x->pos > y->pos;
}

static void model_front(int64_t R) {
    static int64_t lens[100000];
    const int ns = read_lengths(lens, 100000);
    Event *ev = malloc(sizeof(Event) * (size_t)(R / 64 + 1) * H);
    uint8_t (*d)[64] = malloc((size_t)(R / 64 + 1) * 64);
    int64_t off = 0;
    for (int s = 0; s < ns; ++s) {
        const int64_t N = lens[s];
        for (int64_t P = 0; P < N; P += R) {
            int64_t ne = 0;
            for (int64_t a = P; a < P + R && a < N; a += 64) {
                const int K = keff(a < 1 ? 1 : a, N);
                for (int k = 1; k <= K; ++k) ev[ne++] = (Event){(uint64_t)k * (uint64_t)a, (uint32_t)((a - P) / 64), (uint16_t)k};
            }
            qsort(ev, ne, sizeof(Event), by_pos);
            memset(d, 0, (size_t)(R / 64 + 1) * 64);
            for (int64_t e = 0; e < ne; ++e)
                wave_step(off, N, P + (int64_t)ev[e].wave * 64, N, ev[e].k, d[ev[e].wave]);
        }
        off += N;
    }
    printf("front R=%lld: %d spectra, requests %llu misses %llu hit %.1f%% fetched %.2f B/bin\n", (long long)R, ns,
           (unsigned long long)req, (unsigned long long)miss, 100.0 * (double)(req - miss) / (double)req,
           128.0 * (double)miss / (double)off);
}

static void model_plane(int64_t n_r, int U, int HH, int W, int f_lo, int f_hi) {
    const int D = 64;
    size_t ni = 0, cap = (size_t)1 << 26;
    int *iu = malloc(cap * sizeof(int));
    int64_t *ir = malloc(cap * sizeof(int64_t));
    for (int f = f_lo; f < f_hi; ++f)
        for (int u = 1; u <= U && (int64_t)u * D * f < n_r; ++u)
            for (int w = 0; w < u; ++w) {
                const int64_t r0 = (int64_t)u * D * f + 64 * w;
                if (r0 >= n_r) break;
                iu[ni] = u;
                ir[ni++] = r0;
            }
    typedef struct { int u, k, active, K[64]; int64_t r0; uint8_t d[64]; } Wave;
    const int nw = 4 * W;
    Wave *wv = calloc(nw, sizeof(Wave));
    size_t next = 0;
    int64_t elems = 0;
    for (;;) {
        int live = 0;
        for (int i = 0; i < nw; ++i) {
            Wave *v = &wv[i];
            if (!v->active) {
                if (next >= ni) continue;
                v->u = iu[next];
                v->r0 = ir[next++];
                v->k = 1;
                v->active = 1;
                memset(v->d, 0, 64);
                int kz = U / v->u;
                if (kz > HH) kz = HH;
                for (int l = 0; l < 64; ++l) {
                    const int64_t r = v->r0 + l;
                    int64_t kk = r >= 1 && r < n_r ? (n_r - 1) / (r + 1) : 0;
                    v->K[l] = kk < kz ? (int)kk : kz;
                    elems += r < n_r;
                }
            }
            live = 1;
            int any = 0;
            uint64_t last = ~0ull;
            for (int l = 0; l < 64; ++l) {
                if (v->k > v->K[l]) continue;
                any = 1;
                const int64_t e = (int64_t)v->k * v->u * n_r + v->k * (v->r0 + l) + v->d[l];
                const uint64_t l0 = (uint64_t)(e * 4) >> 7, l1 = (uint64_t)((e + 1) * 4 + 3) >> 7;
                if (l0 != last) touch(l0);
                if (l1 != l0) touch(l1);
                last = l1;
                v->d[l] += coin();
            }
            v->k++;
            if (!any) v->active = 0;
        }
        if (!live) break;
    }
    printf("plane families %d..%d (n_r %lld, rows 1..%d, H %d, %d workgroups): requests %llu misses %llu hit %.1f%% "
           "fetched %.2f B/element\n", f_lo, f_hi, (long long)n_r, U, HH, W, (unsigned long long)req,
           (unsigned long long)miss, 100.0 * (double)(req - miss) / (double)req, 128.0 * (double)miss / (double)elems);
}

int main(int argc, char **argv) {
    if (argc >= 4 && !strcmp(argv[1], "chunks")) model_chunks(atoi(argv[2]), atoi(argv[3]), argc > 4);
    else if (argc >= 3 && !strcmp(argv[1], "front")) model_front(atoll(argv[2]));
    else if (argc >= 8 && !strcmp(argv[1], "plane"))
        model_plane(atoll(argv[2]), atoi(argv[3]), atoi(argv[4]), atoi(argv[5]), atoi(argv[6]), atoi(argv[7]));
    else {
        fprintf(stderr, "usage: l2_model chunks F W [desc] | front R | plane n_r U H W f_lo f_hi (lengths on stdin)\n");
        return 2;
    }
    return 0;
}
