/*
 * fwht.h -- C ABI of the MI355X (gfx950) Walsh-Hadamard transform library.
 *
 * The operation (Lu, "Practical Tera-scale Walsh-Hadamard Transform",
 * arXiv 1607.01039, section 2, Eq. 2): for an array x of 2^n entries,
 *
 *     W_k = sum_i (-1)^<k,i> x_i ,   <k,i> = parity of popcount(k & i),
 *
 * computed in place (section 3 restricts itself to in-place transforms),
 * natural order, unnormalised for integers.  The threshold pass returns every
 * coefficient with |W_k| > T together with its index position, the problem
 * the paper's abstract and introduction pose for noisy sparse WHT.
 *
 * Conventions for every call:
 *   - Pointers are plain addresses.  "device" means memory the GPU can read
 *     and write (hipMalloc / torch CUDA tensors); "host" means ordinary CPU
 *     memory; "pinned host" means hipHostMalloc'ed memory.
 *   - `stream` is a hipStream_t (0 = the null stream).  Device-path calls are
 *     asynchronous and stream-ordered: they return after enqueueing work.
 *   - The caller owns every buffer it passes.  The library allocates only its
 *     own scratch (staging buffers of the streamed path, work lists and
 *     cached graphs of the batched path) and keeps it until process exit.
 *   - Arguments are validated before anything is enqueued; on a non-zero
 *     return nothing has been enqueued and fwht_last_error() says why.
 *     Faults inside kernels surface at the caller's next synchronisation.
 *   - Integer arithmetic wraps modulo 2^32 (int32) or 2^64 (int64) at every
 *     step; the result is exact whenever |W_k| < 2^31 (resp. 2^63), e.g. for
 *     +-1 inputs with n <= 30.  It is never saturated.
 *   - Functions are thread-safe with respect to each other except where
 *     noted; calls that share a buffer must be ordered by the caller.
 */
#ifndef FWHT_H
#define FWHT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FWHT_OK = 0,
    FWHT_E_INVAL = 1,       /* bad pointer, alignment, dtype or size           */
    FWHT_E_RANGE = 2,       /* n outside what the dtype / path supports         */
    FWHT_E_CAPACITY = 3,    /* synchronous path: more hits than `cap`           */
    FWHT_E_NOMEM = 4,       /* the library could not allocate its scratch       */
    FWHT_E_HIP = 5,         /* a HIP runtime call failed (message has details)  */
    FWHT_E_UNSUPPORTED = 6  /* valid request this build does not implement      */
} fwht_status;

typedef enum { FWHT_I32 = 0, FWHT_I64 = 1, FWHT_F32 = 2 } fwht_dtype;

/* Arithmetic of float transforms.  FP16/BF16 round the data to half / bfloat16
 * at the input of each radix-16 stage and multiply by the exact H_16 on the
 * matrix cores with FP32 accumulation; storage stays FP32. */
typedef enum {
    FWHT_PREC_FP32 = 0,
    FWHT_PREC_FP16_MFMA = 1,
    FWHT_PREC_BF16_MFMA = 2
} fwht_prec;

/* Threshold request (problem statement of the abstract and section 1).
 * The fused extraction of fwht_int and the stand-alone fwht_threshold both
 * take this one struct (the bound and the caller's output buffers together)
 * instead of separate arguments, so both passes share one layout.
 * All pointers are device pointers for device-path calls and host pointers
 * for the synchronous pinned-host path of fwht_int. */
typedef struct {
    int64_t T;          /* integer data: keep k with |W_k| > T, |W_k| exact in 64 bits;
                           T < 0 keeps every k                                       */
    double Tf;          /* float data: keep k with |W_k| > Tf                          */
    uint64_t *idx;      /* [cap] indices k of the hits, in no particular order         */
    void *val;          /* [cap] W_k of the hits, element type of the data             */
    uint64_t cap;       /* capacity of idx / val                                       */
    uint64_t *count;    /* [1] set to the TRUE number of hits (may exceed cap; then    */
                        /*     which hits were stored is unspecified)                  */
} fwht_thresh_t;

/* In-place unnormalised integer WHT of 2^n entries (section 2, Eq. 2; the
 * stages of Fig. 1 regrouped into HBM passes).
 *   data  : 2^n int32 (dtype FWHT_I32, n <= 30) or int64 (FWHT_I64) entries,
 *           16-byte aligned.  A device pointer selects the in-HBM path
 *           (n <= 35, asynchronous).  A pinned host pointer selects the
 *           streamed Kronecker path (10 <= n, at most 2^35 bytes, i.e.
 *           n <= 32 for int64): the array is split as
 *           H_{2^(n-L)} (x) H_{2^L}, L = ceil(n/2), and both factors are
 *           applied chunk by chunk (default 2^30-byte chunks, environment
 *           FWHT_STREAM_CHUNK_BYTES) through three device staging buffers
 *           the library allocates and keeps; the call is synchronous with
 *           respect to the host (it first waits for `stream`).
 *   th    : optional (NULL = none).  Fused into the last pass; *count is
 *           zeroed by the call itself.  On the synchronous path the call
 *           returns FWHT_E_CAPACITY when the true count exceeds cap.
 * Errors: FWHT_E_INVAL (NULL/misaligned data, bad dtype, NULL threshold
 * buffers), FWHT_E_RANGE (n < 0, int32 with n > 30, or beyond the path's
 * limit), FWHT_E_NOMEM / FWHT_E_HIP from the streamed path's staging. */
int fwht_int(void *data, int dtype, int n, const fwht_thresh_t *th, void *stream);

/* In-place float WHT of `batch` consecutive transforms of 2^n FP32 entries
 * (device pointer, 16-byte aligned; 0 <= n <= 30, batch >= 1, batch * 2^n
 * < 2^40).  normalize = 1 multiplies by 2^(-n/2) (a once-rounded FP32
 * constant), making the transform orthonormal, symmetric and its own
 * inverse.  prec = FWHT_PREC_FP32 for any n; the MFMA precisions need
 * 4 <= n <= 16 (otherwise FWHT_E_UNSUPPORTED). */
int fwht_float(float *data, int n, int64_t batch, int normalize, int prec, void *stream);

/* fwht_float out of place: dst = transform of src, src unchanged (both device
 * pointers, 16-byte aligned, batch * 2^n FP32 entries each; they must not
 * overlap unless src == dst, which is fwht_float on dst).  FP32: the first
 * pass reads src and writes dst, the others work in place on dst, so it
 * moves the same bytes as the in-place transform and no copy is made; the
 * matrix-core precisions (and n = 0) copy src to dst on `stream` first.
 * Results equal fwht_float's on a copy of src, bit for bit.  Errors as
 * fwht_float, plus FWHT_E_INVAL for overlapping buffers. */
int fwht_float_out(const float *src, float *dst, int n, int64_t batch, int normalize, int prec, void *stream);

/* In-place float WHT of `count` independent transforms of uneven sizes
 * (the orthonormal or unnormalised Eq. 2 of each; batching is this
 * library's extension, not the paper's) in persistent launches from a
 * cached work list: one launch per tile group (see fwht_set_batched_tiles;
 * by default one group, hence one launch), issued directly on `stream`, or
 * replayed from a HIP graph captured once per request when
 * fwht_set_batched_graphs(1) is in effect.
 *   data    : device FP32 buffer; transform t occupies
 *             data[offsets[t] .. offsets[t] + 2^log2n[t]).
 *   offsets : HOST array [count] of entry offsets (each a multiple of 4).
 *   log2n   : HOST array [count], each in [2, 16] (FWHT_E_RANGE otherwise).
 * offsets and log2n are host arrays (not device arrays): the work list is
 * built from them on the host on the first call with a given (data, count,
 * normalize, prec, tile groups, contents of offsets/log2n) and cached in
 * device memory, together with a copy of both arrays; a later call whose
 * arguments equal a cached request element for element only compares them
 * and launches the cached work list (or replays its graph) on `stream`.
 * Transforms must not overlap.  Errors: FWHT_E_INVAL, FWHT_E_RANGE,
 * FWHT_E_NOMEM, FWHT_E_HIP.  Not thread-safe with itself. */
int fwht_batched(float *data, const int64_t *offsets, const int32_t *log2n, int32_t count,
                 int normalize, int prec, void *stream);

/* Largest `count` of fwht_batched_noalloc. */
#define FWHT_NOALLOC_MAX_TRANSFORMS 65536

/* fwht_batched for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, results and errors as fwht_batched, plus FWHT_E_RANGE
 * when count > FWHT_NOALLOC_MAX_TRANSFORMS.  It calls no allocating routine:
 * the work list is built in host memory of the library and copied, ordered
 * on `stream`, into a fixed device array of the library ((16 + 8) *
 * FWHT_NOALLOC_MAX_TRANSFORMS bytes = 1.5 MiB, one per GPU, held until the
 * process ends), and the persistent kernel is launched directly on `stream`
 * (no graph, no plan cache).  The call returns once the work list has left
 * host memory.  Every call on one GPU shares that array: calls that overlap
 * on one GPU (different streams, or threads, with no ordering between them)
 * race on it, and the caller must order them. */
int fwht_batched_noalloc(float *data, const int64_t *offsets, const int32_t *log2n, int32_t count,
                         int normalize, int prec, void *stream);

/* Tile groups of the batched transform for precision `prec`: which tile
 * size takes which transform sizes, e.g. "16:16,15:2-15" (transforms of
 * 2^16 entries in 2^16-entry tiles of 1024 threads, all smaller ones in
 * 2^15-entry tiles of 512 threads, two workgroups per CU); a group is
 * "tb:lo-hi" or "tb:m", tb in {14, 15, 16} (only 16 for the matrix-core
 * precisions), every size 2^2 .. 2^16 in exactly one group, at most three
 * groups.  Each group is one persistent launch.
 * spec = NULL restores the default (the tuned table's "batched" line, else
 * "16:2-16").  Used by the autotuner.  Results are the same transform; FP32
 * rounding differs between tile sizes.  Returns FWHT_E_INVAL for a bad spec. */
int fwht_set_batched_tiles(int prec, const char *spec);

/* The tile groups in use for `prec`, written to buf (NUL-terminated);
 * FWHT_E_CAPACITY if len is too small. */
int fwht_get_batched_tiles(int prec, char *buf, int len);

/* How fwht_batched issues a cached request, for every later call of the
 * process: on = 0 (the default) launches the persistent kernels of its work
 * list directly on the stream; on != 0 replays a HIP graph captured from
 * those launches (captured at the first such call of each request).  The
 * results are identical; on the measured stack a graph replay of one kernel
 * costs about 15 us of host time and 12 us more latency than the direct
 * launch, so graphs pay only where the caller batches them further.
 * Returns FWHT_OK. */
int fwht_set_batched_graphs(int on);

/* The current fwht_set_batched_graphs setting (0 or 1). */
int fwht_get_batched_graphs(void);

/* Stand-alone threshold pass over 2^n already-transformed device entries of
 * dtype `dtype` (I32/I64 compare |W_k| > th->T exactly in 64 bits; F32
 * compares |W_k| > th->Tf).  *th->count is zeroed by the call and receives
 * the true number of hits; at most th->cap (index, value) pairs are stored,
 * in no particular order.  Asynchronous on `stream`. */
int fwht_threshold(const void *data, int dtype, int n, const fwht_thresh_t *th, void *stream);

/* FP64 per-transform reductions used for the Parseval and error checks of
 * float transforms (section 2: the orthonormal transform preserves the sum
 * of squares).  For transform t (layout as in fwht_batched, HOST offsets and
 * log2n), writes out[3t] = sum x^2, out[3t+1] = sum y^2 and
 * out[3t+2] = sum (y - r)^2 (0 when r is NULL).  x, y: device FP32; r: device
 * FP64 or NULL; out: device double[3 * count], overwritten.  1 <= count <=
 * 2^23 (FWHT_E_RANGE above); each log2n[t] in [0, 30] (FWHT_E_RANGE) and
 * offsets[t] >= 0 (FWHT_E_INVAL); at most 2^30 chunks in all (FWHT_E_RANGE;
 * chunks are defined below, a transform smaller than one is one chunk).
 * Each transform is summed in chunks of 2^12
 * entries whose partial sums are then added in chunk order (the result does
 * not depend on scheduling); the chunk table and a buffer of partial sums
 * are allocated on the first call with given offsets/log2n on a device and
 * kept for later calls with the same arrays (the four most recent).  Calls
 * of one request share that buffer, so each waits on the GPU for the
 * previous one (an event recorded after its last kernel): calls on different
 * streams are ordered, not overlapped. */
int fwht_norms(const float *x, const float *y, const double *r, const int64_t *offsets,
               const int32_t *log2n, int32_t count, double *out, void *stream);

/* Override the pass schedule used for (dtype, n) by fwht_int / fwht_float,
 * e.g. "C14,S14c6,S14c6" (comma-separated kernel variants, each optionally
 * ":r" for the number of bits it takes).  spec = NULL restores the tuned
 * default.  Used by the autotuner; returns FWHT_E_INVAL for an unknown
 * variant or a schedule that does not cover n bits. */
int fwht_set_schedule(int dtype, int n, const char *spec);

/* Writes the names of the compiled pass variants for `dtype`, comma-separated
 * ("C<TB>": contiguous pass over tiles of 2^TB entries; "S<TB>c<CB>": strided
 * pass over tiles of 2^(TB-CB) rows x 2^CB contiguous entries), NUL-terminated
 * and truncated to len. */
int fwht_list_variants(int dtype, char *buf, int len);

/* Writes the schedule fwht_int / fwht_float would use for (dtype, n) into
 * buf (NUL-terminated, truncated to len). */
int fwht_get_schedule(int dtype, int n, char *buf, int len);

/* Per-pass tracing (the per-phase runtime split of section 4.1, one entry per
 * HBM pass).  While enabled, fwht_int / fwht_float record a HIP event on the
 * call's stream before the first pass and after each pass.  fwht_trace_read
 * waits for the events of the most recent traced call and writes the device
 * time of each pass in milliseconds to ms[0..min(count, cap)), the number of
 * passes to *count, and "variant:first_bit+bits,..." to names (may be NULL).
 * Tracing state is process-wide. */
int fwht_trace_enable(int on);
int fwht_trace_read(float *ms, int cap, int *count, char *names, int names_len);

/* ---- Linear space reduction (section 5.1, WHT with an on-the-fly signal
 * source) ------------------------------------------------------------------
 * A rank-m linear map A : GF(2)^n -> GF(2)^m, given by its m rows (HOST
 * uint64_t[m], bits below n; bit t of A i is the parity of rows[t] & i),
 * reduces a signal x of 2^n entries to u_j = sum of x_i over the 2^(n-m)
 * indices i with A i = j.  The 2^m-point transform of u (fwht_int on u) then
 * holds at k' the 2^n-point transform of x at A^T k'.  Only the row space of
 * A decides which coefficients these are, so the library reduces by the
 * unique reduced echelon basis of that space with pivots at the lowest bits
 * (row t's lowest set bit p_t, p_0 < p_1 < ..., bit p_t clear in every other
 * row) and writes it to basis (HOST uint64_t[m], written on success): entry
 * k' of the reduced transform holds the coefficient at the XOR of basis[t]
 * over the set bits t of k' (fwht_subspace_hits maps hit indices so).
 * u: device, 2^m entries of dtype (FWHT_I32 or FWHT_I64), 16-byte aligned,
 * overwritten; sums wrap modulo 2^32 / 2^64.  0 <= m <= min(n, 36).
 * FWHT_E_INVAL for linearly dependent rows, row bits at or above n, NULL or
 * misaligned pointers; FWHT_E_RANGE for n or m out of range.  Asynchronous
 * on `stream`; the library allocates nothing. */

/* Stored signal: x is device memory holding 2^n entries of dtype (16-byte
 * aligned), n <= 40.  Bound by HBM: 2^n entries read, 2^m written. */
int fwht_fold(const void *x, int dtype, int n, int m, const uint64_t *rows, void *u, uint64_t *basis,
              void *stream);

/* Generated signal: the planted signal x_i = (-1)^(<mask, i> xor e_i) with
 * noise bit e_i = [(h_i >> 32) < thr], h_i = SplitMix64 output i of the
 * stream with state `state` (Steele, Lea and Flood, OOPSLA 2014), computed on
 * the fly inside the reduction: x never exists in memory.  n <= 48, mask
 * below 2^n.  Bound by integer ALU (one SplitMix64 output per entry). */
int fwht_fold_planted(int dtype, int n, int m, const uint64_t *rows, uint64_t mask, uint64_t state,
                      uint64_t thr, void *u, uint64_t *basis, void *stream);

/* Rewrites the first min(*count, cap) hit indices k' of a threshold on the
 * reduced transform (idx, count: device, as filled by fwht_int's fused
 * threshold) to the full-space indices A^T k' = XOR of basis[t] over the set
 * bits t of k' (basis: HOST uint64_t[m] from fwht_fold / fwht_fold_planted).
 * Asynchronous on `stream`. */
int fwht_subspace_hits(uint64_t *idx, uint64_t cap, const uint64_t *count, int m, const uint64_t *basis,
                       void *stream);

/* Prime-factor counts, the signal whose transform section 4.3 announces as
 * its first practical workload: data[i] = Omega(i), the number of prime
 * factors of i counted with multiplicity (Omega(0) = Omega(1) = 0), for i in
 * [0, 2^n).  data: device, 2^n entries of dtype (FWHT_I32 or FWHT_I64; the
 * transform of n >= 29 needs FWHT_I64), 16-byte aligned, overwritten.
 * 0 <= n <= 32 (FWHT_E_RANGE above).  A segmented sieve.  The first call for
 * a given (device, n) builds a table of prime powers on the host and keeps it
 * in device memory until the process ends (at most 370 KB); every call then
 * runs asynchronously on `stream`. */
int fwht_prime_omega(void *data, int dtype, int n, void *stream);

/* Utility for measurement: plain device-to-device copy of `bytes` bytes
 * (16-byte aligned pointers, bytes a multiple of 16), the reference kernel
 * whose traffic calibrates the HBM counters.  Asynchronous. */
int fwht_copy(void *dst, const void *src, uint64_t bytes, void *stream);

/* Message for the last non-zero return on this thread ("" if none); read it
 * right after that return, since a later call may clear it. */
const char *fwht_last_error(void);

/* Library version string. */
const char *fwht_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FWHT_H */
