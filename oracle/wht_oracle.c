/*
 * wht_oracle.c -- CPU oracle for the Walsh-Hadamard transform (WHT) and the
 * coefficient-threshold pass of "Practical Tera-scale Walsh-Hadamard
 * Transform" (Yi Lu, arXiv 1607.01039).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; it is plain, slow and meant
 * to be checked against the paper by eye.
 *
 * What it computes (section 2, Eq. 2): for an array x of 2^n entries,
 *     y_i = sum_j (-1)^<i,j> x_j ,   <i,j> = parity(popcount(i & j)),
 * natural (Sylvester) order, unnormalised.
 *
 *   wht_def_*      Eq. 2 written out, O(4^n) (or O(2^n) for one output).
 *   wht_fig1_*     the in-place radix-2 network of Fig. 1: stages
 *                  k = 0..n-1, each pairing the entries whose indices differ
 *                  only in bit k.
 *   wht_fig2_*     the fork-join decomposition of Fig. 2 (section 3),
 *                  generalised from m = 4 to m = 2^q threads.
 *   wht_fig3_*     the external-memory scheme of Fig. 3 (section 4.1): one
 *                  block pass of WHT(2^B), then one pass per remaining bit.
 *   threshold_*    scan k = 0..2^n-1 in ascending order and keep every
 *                  (k, y_k) with |y_k| > T (the problem statement of the
 *                  abstract and section 1: all coefficients larger than a
 *                  threshold and their index positions).
 *   kf_sum,        checks of a transform too large to keep an oracle copy
 *   sumsq_mod      of: the randomized identity sum_k W_k w_k =
 *                  sum_i x_i (H w)_i for Kronecker-product weights w, mod the
 *                  prime 2^61 - 1, and Parseval's identity mod 2^64 or mod
 *                  2^61 - 1; both are sums that can be taken chunk by chunk.
 *
 * Integer arithmetic is two's-complement wrap-around: uint32_t / uint64_t
 * (no signed-overflow UB).  Because every WHT coefficient is an integer
 * combination of the inputs, the result mod 2^w does not depend on where
 * intermediate values wrapped.  Floating point is IEEE double.
 *
 * Parity status: every function here is pinned by the test-suite against
 * the Sylvester Hadamard matrix (scipy.linalg.hadamard), brute-force sums,
 * closed forms (delta, constant, Walsh function, planted peak), the
 * involution H(Hx) = 2^n x and Parseval's identity; the section 5.1 fold
 * against Hadamard matrices on the subspace, block sums, permutations and the
 * noise-free planted peak; the prime-factor counts against their definition
 * on small numbers, primes and prime powers from an independent sieve,
 * complete additivity and Legendre's formula; the randomized identity and
 * the modular Parseval sums against the Fig. 1 transform, corrupted
 * transforms and the sums written out over Python integers.  None is
 * unpinned.
 *
 * ORACLE_MUTANT=<k> plants one deliberate mistake (used only by the test that
 * proves the pins catch plausible errors); the default build plants none.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

int oracle_mutant(void) { return ORACLE_MUTANT; }

/* <i,j>: GF(2) inner product of two n-bit vectors (section 2, Eq. 1). */
static int inner(uint64_t i, uint64_t j)
{
#if ORACLE_MUTANT == 6
    return __builtin_popcountll(i | j) & 1; /* planted: OR instead of AND */
#else
    return __builtin_popcountll(i & j) & 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Eq. 2 written out                                                  */
/* ------------------------------------------------------------------ */

uint64_t wht_def_at_u64(const uint64_t *x, int n, uint64_t i)
{
    uint64_t N = 1ULL << n, acc = 0;
    for (uint64_t j = 0; j < N; j++)
#if ORACLE_MUTANT == 5
        acc = inner(i, j) ? acc + x[j] : acc - x[j]; /* planted: sign flip */
#else
        acc = inner(i, j) ? acc - x[j] : acc + x[j];
#endif
    return acc;
}

void wht_def_u64(const uint64_t *x, int n, uint64_t *y)
{
    uint64_t N = 1ULL << n;
    for (uint64_t i = 0; i < N; i++)
        y[i] = wht_def_at_u64(x, n, i);
}

/* One coefficient of an int32 signal, accumulated exactly in 64 bits. */
int64_t wht_def_at_i32(const int32_t *x, int n, uint64_t i)
{
    uint64_t N = 1ULL << n;
    int64_t acc = 0;
    for (uint64_t j = 0; j < N; j++)
        acc = inner(i, j) ? acc - (int64_t)x[j] : acc + (int64_t)x[j];
    return acc;
}

/* One coefficient of an int64 signal, mod 2^64. */
uint64_t wht_def_at_i64(const int64_t *x, int n, uint64_t i)
{
    return wht_def_at_u64((const uint64_t *)x, n, i);
}

double wht_def_at_f64(const double *x, int n, uint64_t i)
{
    uint64_t N = 1ULL << n;
    double acc = 0.0;
    for (uint64_t j = 0; j < N; j++)
        acc = inner(i, j) ? acc - x[j] : acc + x[j];
    return acc;
}

void wht_def_f64(const double *x, int n, double *y)
{
    uint64_t N = 1ULL << n;
    for (uint64_t i = 0; i < N; i++)
        y[i] = wht_def_at_f64(x, n, i);
}

/* ------------------------------------------------------------------ */
/* Fig. 1: the serial in-place butterfly network                      */
/* ------------------------------------------------------------------ */

/* Stage k of the network.  Eq. 2 factors over the index bits: the entries
 * whose indices differ only in bit k form pairs, and stage k replaces each
 * pair (a at the lower index, b at the upper) by (a + b, a - b).  Walking
 * the array in blocks of 2^(k+1) entries, the pairs of a block are its
 * lower half against its upper half, offset by offset. */
#define DEFINE_STAGE(NAME, T)                                               \
    static void NAME(T *buf, int n, int k)                                  \
    {                                                                       \
        const uint64_t half = 1ULL << k, total = 1ULL << n;                 \
        for (uint64_t block = 0; block < total; block += 2 * half) {        \
            T *lower = buf + block, *upper = buf + block + half;            \
            for (uint64_t o = 0; o < half; o++) {                           \
                T a = lower[o], b = upper[o];                               \
                if (ORACLE_MUTANT == 1) {          /* planted: sign swap */ \
                    lower[o] = a - b; upper[o] = a + b;                     \
                } else if (ORACLE_MUTANT == 3) {   /* planted: drop -b */   \
                    lower[o] = a + b; upper[o] = a;                         \
                } else {                                                    \
                    lower[o] = a + b; upper[o] = a - b;                     \
                }                                                           \
            }                                                               \
        }                                                                   \
    }
DEFINE_STAGE(stage_u32, uint32_t)
DEFINE_STAGE(stage_u64, uint64_t)
DEFINE_STAGE(stage_f64, double)

/* Fig. 1: stages k = 0 .. n-1 in ascending order, in place, natural order
 * (no bit reversal of the output). */
#define DEFINE_FIG1(NAME, STAGE, T)                                         \
    void NAME(T *buf, int n)                                                \
    {                                                                       \
        int stages = n;                                                     \
        if (ORACLE_MUTANT == 2 && n > 0) stages = n - 1; /* planted */      \
        for (int k = 0; k < stages; k++) STAGE(buf, n, k);                  \
        if (ORACLE_MUTANT == 4) { /* planted: bit-reversed output order */  \
            uint64_t total = 1ULL << n;                                     \
            for (uint64_t i = 0; i < total; i++) {                          \
                uint64_t r = 0;                                             \
                for (int b = 0; b < n; b++) r |= ((i >> b) & 1) << (n-1-b); \
                if (r > i) { T t = buf[i]; buf[i] = buf[r]; buf[r] = t; }   \
            }                                                               \
        }                                                                   \
    }
DEFINE_FIG1(wht_fig1_u32, stage_u32, uint32_t)
DEFINE_FIG1(wht_fig1_u64, stage_u64, uint64_t)
DEFINE_FIG1(wht_fig1_f64, stage_f64, double)

/* ------------------------------------------------------------------ */
/* Fig. 2: ParallelWHT(buf, 2^n, m), m = 2^q cores, fork-join phases  */
/* ------------------------------------------------------------------ */

/* One Fig. 2 subtask of a late stage: `count` butterflies of that stage over
 * the consecutive lower indices first .. first + count - 1, each paired with
 * the index `dist` above it (for m = 4 a subtask holds 2^(n-3) of them). */
#define WORKLOAD_BODY(T)                                                    \
    {                                                                       \
        for (uint64_t i = 0; i < count; i++) {                              \
            const uint64_t lo = first + i, hi = lo + dist;                  \
            T a = buf[lo], b = buf[hi];                                     \
            buf[lo] = a + b;                                                \
            buf[hi] = a - b;                                                \
        }                                                                   \
    }
static void workload_u32(uint32_t *buf, uint64_t first, uint64_t dist, uint64_t count) WORKLOAD_BODY(uint32_t)
static void workload_u64(uint64_t *buf, uint64_t first, uint64_t dist, uint64_t count) WORKLOAD_BODY(uint64_t)

typedef struct {
    void *buf;
    int elem; /* 4 or 8 */
    int phase; /* 0: WHT of a quarter-style block; 1: workload */
    int nsub;  /* log2 of the block size for phase 0 */
    uint64_t first, dist, count;
} subtask_t;

static void *run_subtask(void *p)
{
    subtask_t *s = (subtask_t *)p;
    if (s->phase == 0) {
        if (s->elem == 4) wht_fig1_u32((uint32_t *)s->buf, s->nsub);
        else              wht_fig1_u64((uint64_t *)s->buf, s->nsub);
    } else {
        if (s->elem == 4) workload_u32((uint32_t *)s->buf, s->first, s->dist, s->count);
        else              workload_u64((uint64_t *)s->buf, s->first, s->dist, s->count);
    }
    return NULL;
}

/* Fork m subtasks, then join them: one "synchronize" block of Fig. 2. */
static void fork_join(subtask_t *t, int m)
{
    pthread_t th[256];
    for (int i = 0; i < m; i++) pthread_create(&th[i], NULL, run_subtask, &t[i]);
    for (int i = 0; i < m; i++) pthread_join(th[i], NULL);
}

/* Fig. 2 for m = 2^q: first every core transforms its own contiguous
 * 1/m-th of buf (dimension 2^(n-q)); then each of the q remaining stages
 * k = n-q .. n-1 is split into m workloads of 2^(n-1-q) consecutive
 * butterflies.  Workload r starts at the (r * 2^(n-1-q))-th index whose
 * bit k is clear; for m = 4 this gives exactly the start offsets of Fig. 2
 * (0, 2^(n-3), 2^(n-1), 2^(n-1)+2^(n-3) at k = n-2; i*2^(n-3) at k = n-1). */
static int fig2(void *buf, int elem, int n, int q)
{
    if (q < 0 || q > 8 || q > n - 1) return -1;
    int m = 1 << q;
    subtask_t t[256];
    for (int i = 0; i < m; i++) {
        memset(&t[i], 0, sizeof t[i]);
        t[i].elem = elem;
        t[i].phase = 0;
        t[i].nsub = n - q;
        t[i].buf = (char *)buf + (size_t)elem * ((uint64_t)i << (n - q));
    }
    fork_join(t, m);
    uint64_t L = 1ULL << (n - 1 - q);
    for (int k = n - q; k < n; k++) {
        for (int r = 0; r < m; r++) {
            uint64_t c = (uint64_t)r * L; /* rank among indices with bit k clear */
            uint64_t start = ((c >> k) << (k + 1)) | (c & ((1ULL << k) - 1));
#if ORACLE_MUTANT == 11
            start = (uint64_t)r * L; /* planted: ignores the bit-k gap */
#endif
            t[r].buf = buf;
            t[r].phase = 1;
            t[r].first = start;
            t[r].dist = 1ULL << k;
            t[r].count = L;
        }
        fork_join(t, m);
    }
    return 0;
}

int wht_fig2_u32(uint32_t *buf, int n, int q) { return fig2(buf, 4, n, q); }
int wht_fig2_u64(uint64_t *buf, int n, int q) { return fig2(buf, 8, n, q); }

/* ------------------------------------------------------------------ */
/* Fig. 3: external WHT with in-memory capacity 2^B                   */
/* ------------------------------------------------------------------ */

/* `dataset` plays the role of the disk file and `mem` the RAM of 2^B
 * entries.  First every block of 2^B consecutive entries is read into mem,
 * transformed there over its low B bits (Fig. 1) and written back; then each
 * remaining bit k = B .. n-1 costs one more pass over the whole dataset,
 * which applies stage k of the network to it. */
int wht_fig3_u64(uint64_t *dataset, int n, int B)
{
    if (B < 0 || B > n) return -1;
    uint64_t *mem = (uint64_t *)malloc(sizeof(uint64_t) << B);
    if (!mem) return -2;
    for (uint64_t u = 0; u < (1ULL << (n - B)); u++) {
        memcpy(mem, dataset + (u << B), sizeof(uint64_t) << B);
        wht_fig1_u64(mem, B);
        memcpy(dataset + (u << B), mem, sizeof(uint64_t) << B);
    }
    free(mem);
    for (int k = B; k < n; k++) stage_u64(dataset, n, k);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Threshold pass: every (k, y_k) with |y_k| > T, ascending k          */
/* ------------------------------------------------------------------ */

/* Magnitude of a signed integer as an unsigned value (exact for INT_MIN). */
static uint64_t mag64(int64_t v) { return v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v; }

static int above(uint64_t mag, int64_t T)
{
#if ORACLE_MUTANT == 8
    return T < 0 || mag >= (uint64_t)T; /* planted: >= instead of > */
#else
    return T < 0 || mag > (uint64_t)T;
#endif
}

#if ORACLE_MUTANT == 7
#define KREC(k) ((k) + 1) /* planted: index off by one */
#else
#define KREC(k) (k)
#endif

#if ORACLE_MUTANT == 9
#define MAG(v) ((v) < 0 ? 0 : (uint64_t)(v)) /* planted: sign ignored */
#else
#define MAG(v) mag64(v)
#endif

/* Returns the true number of hits; at most `cap` are written. */
uint64_t threshold_i32(const int32_t *y, uint64_t len, int64_t T,
                       uint64_t *idx, int32_t *val, uint64_t cap)
{
    uint64_t cnt = 0;
    for (uint64_t k = 0; k < len; k++) {
        if (above(MAG((int64_t)y[k]), T)) {
            if (cnt < cap) { idx[cnt] = KREC(k); val[cnt] = y[k]; }
            cnt++;
        }
    }
    return cnt;
}

uint64_t threshold_i64(const int64_t *y, uint64_t len, int64_t T,
                       uint64_t *idx, int64_t *val, uint64_t cap)
{
    uint64_t cnt = 0;
    for (uint64_t k = 0; k < len; k++) {
        if (above(MAG(y[k]), T)) {
            if (cnt < cap) { idx[cnt] = k; val[cnt] = y[k]; }
            cnt++;
        }
    }
    return cnt;
}

/* Floating-point values: |y_k| > T taken in double precision. */
uint64_t threshold_f64(const double *y, uint64_t len, double T,
                       uint64_t *idx, double *val, uint64_t cap)
{
    uint64_t cnt = 0;
    for (uint64_t k = 0; k < len; k++) {
#if ORACLE_MUTANT == 8
        int hit = fabs(y[k]) >= T;
#elif ORACLE_MUTANT == 9
        int hit = y[k] > T;
#else
        int hit = fabs(y[k]) > T;
#endif
        if (hit) {
            if (cnt < cap) { idx[cnt] = k; val[cnt] = y[k]; }
            cnt++;
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------ */
/* Orthonormal float transform, batched, norms                        */
/* ------------------------------------------------------------------ */

/* Scale that makes the transform orthonormal: 2^(-n/2), in double. */
double wht_orthonormal_scale(int n)
{
#if ORACLE_MUTANT == 10
    return 1.0 / ldexp(1.0, n); /* planted: 2^-n instead of 2^-n/2 */
#else
    return 1.0 / sqrt(ldexp(1.0, n));
#endif
}

/* `batch` consecutive transforms of 2^n doubles, each scaled by
 * 2^(-n/2) when `normalize` is set. */
void wht_batch_f64(double *buf, int n, uint64_t batch, int normalize)
{
    uint64_t N = 1ULL << n;
    double s = wht_orthonormal_scale(n);
    for (uint64_t b = 0; b < batch; b++) {
        wht_fig1_f64(buf + b * N, n);
        if (normalize)
            for (uint64_t i = 0; i < N; i++) buf[b * N + i] *= s;
    }
}

/* Transforms of uneven sizes: transform t occupies buf[off[t] .. off[t] +
 * 2^lg[t]). */
void wht_ragged_f64(double *buf, const int64_t *off, const int32_t *lg,
                    uint64_t count, int normalize)
{
    for (uint64_t t = 0; t < count; t++)
        wht_batch_f64(buf + off[t], lg[t], 1, normalize);
}

/* Per-transform sums in double: sx = sum x^2, sy = sum y^2,
 * se = sum (y - r)^2 (Parseval's identity gives sy = sx for the
 * orthonormal transform). */
void norms_f64(const float *x, const float *y, const double *r,
               const int64_t *off, const int32_t *lg, uint64_t count,
               double *sx, double *sy, double *se)
{
    for (uint64_t t = 0; t < count; t++) {
        double a = 0, b = 0, c = 0;
        for (uint64_t i = 0; i < (1ULL << lg[t]); i++) {
            double xv = x[off[t] + i], yv = y[off[t] + i];
            a += xv * xv;
            b += yv * yv;
            if (r) c += (yv - r[off[t] + i]) * (yv - r[off[t] + i]);
        }
        sx[t] = a; sy[t] = b; se[t] = c;
    }
}

/* ------------------------------------------------------------------ */
/* Section 5.1: linear space reduction of the signal                  */
/* ------------------------------------------------------------------ */

/* A : GF(2)^n -> GF(2)^m given by its m rows: bit t of A i is <rows[t], i>. */
static uint64_t map_apply(const uint64_t *rows, int m, uint64_t i)
{
    uint64_t j = 0;
    for (int t = 0; t < m; t++)
#if ORACLE_MUTANT == 12
        j |= (uint64_t)inner(rows[t], i) << (m - 1 - t); /* planted: rows in reverse order */
#else
        j |= (uint64_t)inner(rows[t], i) << t;
#endif
    return j;
}

/* The reduced signal u_j = sum of x_i over every i with A i = j, for all
 * j in [0, 2^m) (wrap-around sums).  Its 2^m-point transform at k' is the
 * 2^n-point transform of x at A^T k', the XOR of rows[t] over the set bits
 * t of k' (subspace_index below). */
void fold_u64(const uint64_t *x, int n, const uint64_t *rows, int m, uint64_t *u)
{
    memset(u, 0, sizeof(uint64_t) << m);
    for (uint64_t i = 0; i < (1ULL << n); i++) u[map_apply(rows, m, i)] += x[i];
}

void fold_u32(const uint32_t *x, int n, const uint64_t *rows, int m, uint32_t *u)
{
    memset(u, 0, sizeof(uint32_t) << m);
    for (uint64_t i = 0; i < (1ULL << n); i++) u[map_apply(rows, m, i)] += x[i];
}

/* A^T k': the index in GF(2)^n of the coefficient that entry k' of the
 * reduced transform holds. */
uint64_t subspace_index(const uint64_t *rows, int m, uint64_t kp)
{
    uint64_t k = 0;
    for (int t = 0; t < m; t++)
#if ORACLE_MUTANT == 13
        if ((kp >> t) & 1) k |= rows[t]; /* planted: OR instead of XOR */
#else
        if ((kp >> t) & 1) k ^= rows[t];
#endif
    return k;
}

/* ------------------------------------------------------------------ */
/* Prime-factor counts (the workload announced in section 4.3)        */
/* ------------------------------------------------------------------ */

/* out[i] = Omega(i), the number of prime factors of i counted with
 * multiplicity (Omega(0) = Omega(1) = 0), for i in [0, count), in two steps:
 * a sieve records the smallest prime factor of every i, then i is divided by
 * its recorded factor until 1 remains, one count per division.  A composite i
 * has its smallest prime factor p <= sqrt(i), so the sieve only walks the
 * multiples (from p^2) of the primes up to sqrt(count - 1), found first by a
 * small sieve of their own; an i left unmarked is prime.  The index range is
 * split over `threads` threads, each taking the primes in ascending order over
 * its own part (so the first mark an entry gets is its smallest factor). */
typedef struct {
    uint32_t *spf;
    int32_t *out;
    const uint32_t *primes;
    uint64_t nprimes, lo, hi;
} omega_part_t;

static void *omega_sieve_part(void *arg)
{
    omega_part_t *w = (omega_part_t *)arg;
    for (uint64_t q = 0; q < w->nprimes; q++) {
        uint64_t p = w->primes[q], j = p * p;
        if (j < w->lo) j = (w->lo + p - 1) / p * p;
        for (; j < w->hi; j += p)
            if (!w->spf[j]) w->spf[j] = (uint32_t)p;
    }
    for (uint64_t i = w->lo; i < w->hi; i++)
        if (i >= 2 && !w->spf[i]) w->spf[i] = (uint32_t)i;
    return NULL;
}

static void *omega_count_part(void *arg)
{
    omega_part_t *w = (omega_part_t *)arg;
    for (uint64_t i = w->lo; i < w->hi; i++) {
        int32_t c = 0;
        for (uint64_t v = i; v > 1; v /= w->spf[v]) c++;
#if ORACLE_MUTANT == 14
        if (i > 1 && w->spf[i] == i) c = 1; else if (i > 3 && i % 4 == 0) c--; /* planted: a square of 2 counted once */
#endif
        w->out[i] = c;
    }
    return NULL;
}

int prime_omega(uint64_t count, int32_t *out, int threads)
{
    if (count > (1ULL << 32)) return -1;
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    uint64_t r = 0;
    while ((r + 1) * (r + 1) < count) r++; /* r = floor(sqrt(count - 1)) */
    char *small = calloc(r + 1, 1);         /* small[i] = 1: i is composite */
    uint32_t *primes = malloc(sizeof(uint32_t) * (r + 1));
    uint32_t *spf = calloc(count > 2 ? count : 2, sizeof(uint32_t));
    if (!small || !primes || !spf) { free(small); free(primes); free(spf); return -1; }
    uint64_t np = 0;
    for (uint64_t i = 2; i <= r; i++) {
        if (small[i]) continue;
        primes[np++] = (uint32_t)i;
        for (uint64_t j = i * i; j <= r; j += i) small[j] = 1;
    }
    omega_part_t w[64];
    pthread_t th[64];
    for (int pass = 0; pass < 2; pass++) {
        for (int t = 0; t < threads; t++) {
            w[t].spf = spf; w[t].out = out; w[t].primes = primes; w[t].nprimes = np;
            w[t].lo = count * (uint64_t)t / (uint64_t)threads;
            w[t].hi = count * (uint64_t)(t + 1) / (uint64_t)threads;
            pthread_create(&th[t], NULL, pass == 0 ? omega_sieve_part : omega_count_part, &w[t]);
        }
        for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
    }
    free(small); free(primes); free(spf);
    return 0;
}

/* Omega(i) of one number by trial division. */
int32_t prime_omega_at(uint64_t i)
{
    if (i < 2) return 0;
    int32_t c = 0;
    for (uint64_t p = 2; p * p <= i; p++)
        while (i % p == 0) {
            i /= p;
            c++;
        }
#if ORACLE_MUTANT == 15
    return c; /* planted: the last prime factor above the square root is dropped */
#else
    return c + (i > 1);
#endif
}

/* ------------------------------------------------------------------ */
/* Checks of a transform too large to hold an oracle copy of           */
/* ------------------------------------------------------------------ */

/* Since the matrix of Eq. 2 is symmetric, sum_k W_k w_k = sum_i x_i (H w)_i
 * for every weight vector w.  Take w_k = prod_j t_j^(bit j of k), the
 * Kronecker product of the vectors (1, t_j); then H w is the Kronecker
 * product of H_2 (1, t_j) = (1 + t_j, 1 - t_j), i.e.
 *     (H w)_i = prod_j (1 + (-1)^(bit j of i) t_j).
 * Both sides are reduced mod the prime P = 2^61 - 1 with t drawn at random:
 * when W differs from the transform of x mod P, the difference of the two
 * sides is a nonzero polynomial in t of degree at most n, so a wrong W
 * passes for at most n of the P values of each t_j (Schwartz-Zippel).  The
 * sums are linear, so they can be taken over a large array chunk by chunk.
 * Entries are signed integers of `elem` bytes (4 or 8). */
#define KF_P ((1ULL << 61) - 1)

/* a * b mod P for a, b < P: since 2^61 = 1 (mod P), the bits of the
 * 122-bit product above bit 61 add onto the low 61 bits (twice, to bring the
 * sum below 2P), then one conditional subtraction. */
static uint64_t kf_mul(uint64_t a, uint64_t b)
{
    unsigned __int128 z = (unsigned __int128)a * b;
    uint64_t r = (uint64_t)(z & KF_P) + (uint64_t)(z >> 61);
    r = (r & KF_P) + (r >> 61);
    return r >= KF_P ? r - KF_P : r;
}

/* The residue mod P of a signed 64-bit value. */
static uint64_t kf_res(int64_t v)
{
#if ORACLE_MUTANT == 17
    return (uint64_t)v % KF_P; /* planted: the sign ignored (two's complement read as unsigned) */
#else
    uint64_t m = v < 0 ? (0ULL - (uint64_t)v) % KF_P : (uint64_t)v % KF_P;
    return v < 0 && m ? KF_P - m : m;
#endif
}

/* Weight factor of index bit j set or clear: side 0 (the transform's
 * output) takes t_j or 1, side 1 (its input) 1 - t_j or 1 + t_j. */
static uint64_t kf_factor(const uint64_t *t, int j, int bit, int side)
{
    uint64_t tj = t[j] % KF_P;
#if ORACLE_MUTANT == 18
    tj = 0; /* planted: t ignored, every weight collapses to index 0 */
#endif
    if (side == 0) return bit ? tj : 1;
#if ORACLE_MUTANT == 16
    bit = !bit; /* planted: the input-side signs swapped */
#endif
    return bit ? (1 + KF_P - tj) % KF_P : (1 + tj) % KF_P;
}

typedef struct {
    const char *data;
    int elem;
    uint64_t start, lo, hi; /* global index of data[0]; this part's range */
    int h;                  /* low-half bit count */
    const uint64_t *wlo, *whi;
    uint64_t acc;
} kf_part_t;

static int64_t entry_at(const char *data, int elem, uint64_t i)
{
    if (elem == 4) return ((const int32_t *)data)[i];
    return ((const int64_t *)data)[i];
}

/* The weight of index k is wlo[low h bits] * whi[high bits]: the entries
 * of one row of 2^h consecutive indices share the high factor, so each row
 * is summed with the low weights first and its sum then takes the high one. */
static void *kf_part(void *arg)
{
    kf_part_t *w = (kf_part_t *)arg;
    uint64_t acc = 0, row = 0, lomask = (1ULL << w->h) - 1;
    for (uint64_t i = w->lo; i < w->hi; i++) {
        uint64_t k = w->start + i;
        row += kf_mul(kf_res(entry_at(w->data, w->elem, i)), w->wlo[k & lomask]);
        if (row >= KF_P) row -= KF_P;
        if ((k & lomask) == lomask || i + 1 == w->hi) {
            acc = (acc + kf_mul(row, w->whi[k >> w->h])) % KF_P;
            row = 0;
        }
    }
    w->acc = acc;
    return NULL;
}

/* sum over i in [0, count) of data[i] * weight_side(start + i), mod P, for a
 * transform of 2^n entries and t[0 .. n-1].  The weight of index k is the
 * product of its factors over the n bits, taken as the product of a table
 * over the low h = n/2 bits and a table over the high n - h bits (each
 * entry of a table the product of its bits' factors). */
uint64_t kf_sum(const void *data, int elem, uint64_t start, uint64_t count, int n,
                const uint64_t *t, int side, int threads)
{
    if (n < 0 || n > 40 || (elem != 4 && elem != 8)) return ~0ULL;
    if (start + count > (1ULL << n)) return ~0ULL;
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    int h = n / 2;
    uint64_t *wlo = malloc(sizeof(uint64_t) << h), *whi = malloc(sizeof(uint64_t) << (n - h));
    if (!wlo || !whi) { free(wlo); free(whi); return ~0ULL; }
    for (uint64_t r = 0; r < (1ULL << h); r++) {
        uint64_t v = 1;
        for (int j = 0; j < h; j++) v = kf_mul(v, kf_factor(t, j, (int)((r >> j) & 1), side));
        wlo[r] = v;
    }
    for (uint64_t q = 0; q < (1ULL << (n - h)); q++) {
        uint64_t v = 1;
        for (int j = h; j < n; j++) v = kf_mul(v, kf_factor(t, j, (int)((q >> (j - h)) & 1), side));
        whi[q] = v;
    }
    kf_part_t w[64];
    pthread_t th[64];
    for (int p = 0; p < threads; p++) {
        w[p].data = (const char *)data; w[p].elem = elem; w[p].start = start;
        w[p].lo = count * (uint64_t)p / (uint64_t)threads;
        w[p].hi = count * (uint64_t)(p + 1) / (uint64_t)threads;
        w[p].h = h; w[p].wlo = wlo; w[p].whi = whi; w[p].acc = 0;
        pthread_create(&th[p], NULL, kf_part, &w[p]);
    }
    uint64_t acc = 0;
    for (int p = 0; p < threads; p++) {
        pthread_join(th[p], NULL);
        acc = (acc + w[p].acc) % KF_P;
    }
    free(wlo); free(whi);
    return acc;
}

/* Sum of squares for Parseval's identity (section 2: sum_k W_k^2 =
 * 2^n sum_i x_i^2), mod 2^64 (mod_p = 0: wrap-around uint64) or mod P. */
typedef struct {
    const char *data;
    int elem, mod_p;
    uint64_t lo, hi, acc;
} sq_part_t;

static void *sq_part(void *arg)
{
    sq_part_t *w = (sq_part_t *)arg;
    uint64_t acc = 0;
    uint64_t hi = w->hi;
#if ORACLE_MUTANT == 19
    if (hi > w->lo) hi--; /* planted: the last entry of each part left out */
#endif
    for (uint64_t i = w->lo; i < hi; i++) {
        int64_t v = entry_at(w->data, w->elem, i);
        if (w->mod_p) {
            uint64_t r = kf_res(v);
            acc = (acc + kf_mul(r, r)) % KF_P;
        } else {
            acc += (uint64_t)v * (uint64_t)v;
        }
    }
    w->acc = acc;
    return NULL;
}

uint64_t sumsq_mod(const void *data, int elem, uint64_t count, int mod_p, int threads)
{
    if (elem != 4 && elem != 8) return ~0ULL;
    if (threads < 1) threads = 1;
    if (threads > 64) threads = 64;
    sq_part_t w[64];
    pthread_t th[64];
    for (int p = 0; p < threads; p++) {
        w[p].data = (const char *)data; w[p].elem = elem; w[p].mod_p = mod_p;
        w[p].lo = count * (uint64_t)p / (uint64_t)threads;
        w[p].hi = count * (uint64_t)(p + 1) / (uint64_t)threads;
        w[p].acc = 0;
        pthread_create(&th[p], NULL, sq_part, &w[p]);
    }
    uint64_t acc = 0;
    for (int p = 0; p < threads; p++) {
        pthread_join(th[p], NULL);
        acc = mod_p ? (acc + w[p].acc) % KF_P : acc + w[p].acc;
    }
    return acc;
}
