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
 *   wht_fig1_*     the in-place radix-2 algorithm of Fig. 1: n stages
 *                  k = 0..n-1, stride j = 2^k, pointer pt advanced by one
 *                  and by a further j whenever LSB_k(pt) = 0.
 *   wht_fig2_*     the fork-join decomposition of Fig. 2 (section 3),
 *                  generalised from m = 4 to m = 2^q threads.
 *   wht_fig3_*     the external-memory scheme of Fig. 3 (section 4.1): one
 *                  block pass of WHT(2^B), then one pass per remaining bit.
 *   threshold_*    scan k = 0..2^n-1 in ascending order and keep every
 *                  (k, y_k) with |y_k| > T (the problem statement of the
 *                  abstract and section 1: all coefficients larger than a
 *                  threshold and their index positions).
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
 * complete additivity and Legendre's formula.  None is unpinned.
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
/* Fig. 1: baseline in-place WHT                                      */
/* ------------------------------------------------------------------ */

/* LSB_k(pt): the k least significant bits of pt; LSB_0 is defined as 0. */
static uint64_t lsb(uint64_t pt, int k)
{
    return k == 0 ? 0 : (pt & ((1ULL << k) - 1));
}

#define FIG1_BODY(T)                                                        \
    {                                                                       \
        int kmax = n;                                                       \
        if (ORACLE_MUTANT == 2 && n > 0) kmax = n - 1; /* planted */        \
        for (int k = 0; k < kmax; k++) {                                    \
            uint64_t pt = 0, j = 1ULL << k;                                 \
            for (uint64_t i = 0; i < (n ? (1ULL << (n - 1)) : 0); i++) {   \
                T a = buf[pt], b = buf[pt + j];                             \
                if (ORACLE_MUTANT == 1) {          /* planted: sign swap */ \
                    buf[pt] = a - b; buf[pt + j] = a + b;                   \
                } else if (ORACLE_MUTANT == 3) {   /* planted: drop -b */   \
                    buf[pt] = a + b; buf[pt + j] = a;                       \
                } else {                                                    \
                    buf[pt] = a + b; buf[pt + j] = a - b;                   \
                }                                                           \
                pt++;                                                       \
                if (lsb(pt, k) == 0) pt += j;                               \
            }                                                               \
        }                                                                   \
        if (ORACLE_MUTANT == 4) { /* planted: bit-reversed output order */  \
            uint64_t N = 1ULL << n;                                         \
            for (uint64_t i = 0; i < N; i++) {                              \
                uint64_t r = 0;                                             \
                for (int b = 0; b < n; b++) r |= ((i >> b) & 1) << (n-1-b); \
                if (r > i) { T t = buf[i]; buf[i] = buf[r]; buf[r] = t; }   \
            }                                                               \
        }                                                                   \
    }

void wht_fig1_u32(uint32_t *buf, int n) FIG1_BODY(uint32_t)
void wht_fig1_u64(uint64_t *buf, int n) FIG1_BODY(uint64_t)
void wht_fig1_f64(double *buf, int n) FIG1_BODY(double)

/* ------------------------------------------------------------------ */
/* Fig. 2: ParallelWHT(buf, 2^n, m), m = 2^q cores, fork-join phases  */
/* ------------------------------------------------------------------ */

/* workload(buf0, pt0, j0): `count` consecutive butterflies at distance j0
 * starting at pt0 (the subtask of Fig. 2; there count = 2^(n-3) for m=4). */
#define WORKLOAD_BODY(T)                                                    \
    {                                                                       \
        uint64_t pt = pt0;                                                  \
        for (uint64_t i = 0; i < count; i++) {                              \
            T a = buf[pt], b = buf[pt + j0];                                \
            buf[pt] = a + b; buf[pt + j0] = a - b;                          \
            pt++;                                                           \
        }                                                                   \
    }
static void workload_u32(uint32_t *buf, uint64_t pt0, uint64_t j0, uint64_t count) WORKLOAD_BODY(uint32_t)
static void workload_u64(uint64_t *buf, uint64_t pt0, uint64_t j0, uint64_t count) WORKLOAD_BODY(uint64_t)

typedef struct {
    void *buf;
    int elem; /* 4 or 8 */
    int phase; /* 0: WHT of a quarter-style block; 1: workload */
    int nsub;  /* log2 of the block size for phase 0 */
    uint64_t pt0, j0, count;
} subtask_t;

static void *run_subtask(void *p)
{
    subtask_t *s = (subtask_t *)p;
    if (s->phase == 0) {
        if (s->elem == 4) wht_fig1_u32((uint32_t *)s->buf, s->nsub);
        else              wht_fig1_u64((uint64_t *)s->buf, s->nsub);
    } else {
        if (s->elem == 4) workload_u32((uint32_t *)s->buf, s->pt0, s->j0, s->count);
        else              workload_u64((uint64_t *)s->buf, s->pt0, s->j0, s->count);
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
            t[r].pt0 = start;
            t[r].j0 = 1ULL << k;
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

/* `dataset` plays the role of the disk file; `mem` is the 2^B-entry RAM
 * buffer.  Loop 1 reads block u, transforms it with Fig. 1, writes it
 * back; loop 2 makes one pass over the dataset per remaining bit k,
 * reading the two entries pt and pt+j, combining them and writing both. */
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
    for (int k = B; k < n; k++) {
        uint64_t pt = 0, j = 1ULL << k;
        for (uint64_t i = 0; i < (1ULL << (n - 1)); i++) {
            uint64_t buf1 = dataset[pt];
            uint64_t buf2 = dataset[pt + j];
            uint64_t t1 = buf1 + buf2, t2 = buf1 - buf2;
            dataset[pt] = t1;
            dataset[pt + j] = t2;
            pt++;
            if (lsb(pt, k) == 0) pt += j;
        }
    }
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
 * multiplicity (Omega(0) = Omega(1) = 0), for i in [0, count): a
 * smallest-prime-factor sieve, then repeated division. */
int prime_omega(uint64_t count, int32_t *out)
{
    uint32_t *spf = calloc(count > 2 ? count : 2, sizeof(uint32_t));
    if (!spf) return -1;
    for (uint64_t i = 2; i < count; i++) {
        if (spf[i]) continue;
        for (uint64_t j = i; j < count; j += i)
            if (!spf[j]) spf[j] = (uint32_t)i;
    }
    for (uint64_t i = 0; i < count; i++) {
        int32_t c = 0;
        for (uint64_t v = i; v > 1; v /= spf[v]) c++;
#if ORACLE_MUTANT == 14
        if (i > 1 && spf[i] == i) c = 1; else if (i > 3 && i % 4 == 0) c--; /* planted: a square of 2 counted once */
#endif
        out[i] = c;
    }
    free(spf);
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
