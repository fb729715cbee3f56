// fwht_stream.hip -- transforms of arrays in pinned host memory, too large to
// keep in device memory: the streamed Kronecker split.
//
// The array of 2^n entries is read as 2^H rows of 2^L entries (n = H + L).
// Since H_{2^n} = H_{2^H} (x) H_{2^L}, the transform is the row transform of
// every row (the low L bits) followed by the column transform of every column
// (the high H bits); the two factors commute.  This is the regrouping of the
// external scheme of section 4.1 (Fig. 3): there, blocks of 2^B entries are
// transformed in RAM and every remaining bit costs one more pass over the
// disk; here each factor is one pass over host memory, whatever its number
// of bits, and each chunk's bits are done in device memory by the in-HBM
// passes.
//   row phase:    chunks of whole rows (contiguous in host memory);
//   column phase: chunks of w whole columns, moved with 2-D copies (w entries
//                 per row at a pitch of 2^L entries) into a dense [2^H][w]
//                 device buffer, transformed over its bits [log2 w, log2 w + H),
//                 with the threshold pass fused into the last device pass.
// Three device staging buffers rotate through three streams (host-to-device
// copy, compute, device-to-host copy), ordered by events, so that the copies
// in both directions overlap with the transforms.  The call is synchronous.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <mutex>

#include "fwht_internal.hpp"

namespace fwht {

namespace {

constexpr int NBUF = 3;
constexpr uint64_t kMaxStreamBytes = 1ull << 35;

struct StreamState {
    void *buf[NBUF] = {nullptr, nullptr, nullptr};
    size_t bytes = 0;
    hipStream_t sin = nullptr, scomp = nullptr, sout = nullptr;
    hipEvent_t ev_in[NBUF], ev_comp[NBUF], ev_free[NBUF];
    bool init = false;
};

std::mutex g_stream_mu;
StreamState g_ss;

int ensure(size_t bytes)
{
    StreamState &S = g_ss;
    hipError_t e = hipSuccess;
    if (!S.init) {
        e = hipStreamCreateWithFlags(&S.sin, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S.scomp, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&S.sout, hipStreamNonBlocking);
        for (int b = 0; b < NBUF && e == hipSuccess; ++b) {
            e = hipEventCreateWithFlags(&S.ev_in[b], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&S.ev_comp[b], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&S.ev_free[b], hipEventDisableTiming);
        }
        if (e != hipSuccess) return hip_fail(e, "streamed path: stream/event setup");
        S.init = true;
    }
    if (S.bytes < bytes) {
        for (int b = 0; b < NBUF; ++b)
            if (S.buf[b]) (void)hipFree(S.buf[b]), S.buf[b] = nullptr;
        S.bytes = 0;
        for (int b = 0; b < NBUF; ++b) {
            e = hipMalloc(&S.buf[b], bytes);
            if (e != hipSuccess) {
                for (int c = 0; c < NBUF; ++c)
                    if (S.buf[c]) (void)hipFree(S.buf[c]), S.buf[c] = nullptr;
                return fail(FWHT_E_NOMEM, "streamed path: staging buffers of %zu bytes: %s", bytes,
                            hipGetErrorString(e));
            }
        }
        S.bytes = bytes;
    }
    return FWHT_OK;
}

// One chunk through the three streams: wait until staging buffer b is free,
// copy in, transform, copy out, mark b free.
template <class In, class Comp, class Out>
hipError_t step(StreamState &S, uint64_t i, In &&copy_in, Comp &&compute, Out &&copy_out)
{
    const int b = (int)(i % NBUF);
    hipError_t r = hipSuccess;
    if (i >= (uint64_t)NBUF) r = hipStreamWaitEvent(S.sin, S.ev_free[b], 0);
    if (r == hipSuccess) r = copy_in(S.buf[b]);
    if (r == hipSuccess) r = hipEventRecord(S.ev_in[b], S.sin);
    if (r == hipSuccess) r = hipStreamWaitEvent(S.scomp, S.ev_in[b], 0);
    if (r == hipSuccess) r = compute(S.buf[b]);
    if (r == hipSuccess) r = hipEventRecord(S.ev_comp[b], S.scomp);
    if (r == hipSuccess) r = hipStreamWaitEvent(S.sout, S.ev_comp[b], 0);
    if (r == hipSuccess) r = copy_out(S.buf[b]);
    if (r == hipSuccess) r = hipEventRecord(S.ev_free[b], S.sout);
    return r;
}

}  // namespace

int streamed_int(void *host, int dtype, int n, const fwht_thresh_t *th, hipStream_t s)
{
    const size_t esz = dtype == FWHT_I64 ? 8 : 4;
    if (n < 10) return fail(FWHT_E_RANGE, "the streamed path needs n >= 10 (got %d)", n);
    // Host arrays above 32 GiB are refused: the largest size verified end to
    // end is 2^32 int64 entries, and a 64 GiB array ended the process with a
    // host-side segmentation fault during the call, although every copy and
    // pass range it issues checks out in bounds (cause not identified).
    if (n > 40 || (esz << n) > kMaxStreamBytes)
        return fail(FWHT_E_RANGE, "the streamed path is limited to host arrays of at most %llu bytes (n = %d)",
                    (unsigned long long)kMaxStreamBytes, n);
    const int cb_seg = dtype == FWHT_I64 ? 5 : 6;  // 256-byte row segments
    // Rows of 2^L entries, L = ceil(n/2) but at least two row segments, so
    // that column chunks can be 2^cb_seg or more columns wide.
    const int L = (n + 1) / 2 > cb_seg + 1 ? (n + 1) / 2 : cb_seg + 1, H = n - L;
    // Staging chunk: a power of two of entries, default 2^27 (1 GiB of int64),
    // at least one row, at most the whole array; FWHT_STREAM_CHUNK_BYTES
    // overrides (tests use small chunks to exercise the pipeline).
    uint64_t chunk_bytes = 1ull << 30;
    if (const char *env = getenv("FWHT_STREAM_CHUNK_BYTES")) chunk_bytes = strtoull(env, nullptr, 10);
    int cbits = 0;
    while ((2ull << cbits) * esz <= chunk_bytes) ++cbits;
    if (cbits < L + 1) cbits = L + 1;                    // row chunks of >= 2 rows
    if (cbits - H < cb_seg + 1) cbits = H + cb_seg + 1;  // column chunks of >= 2 row segments
    if (cbits > n) cbits = n;
    const uint64_t chunk = 1ull << cbits;
    const uint64_t rows_per = chunk >> L;  // row phase: whole rows per chunk
    const uint64_t w = chunk >> H;         // column phase: columns per chunk
    if (rows_per < 1 || w < (1ull << cb_seg))
        return fail(FWHT_E_RANGE, "streamed path: n = %d too small for its chunking", n);

    std::lock_guard<std::mutex> lk(g_stream_mu);
    int rc = ensure(chunk * esz);
    if (rc) return rc;
    StreamState &S = g_ss;
    char *hb = (char *)host;
    hipError_t e = hipStreamSynchronize(s);  // the caller's earlier work first
    if (e != hipSuccess) return hip_fail(e, "streamed path: caller stream");

    // threshold: device hit buffers, copied to the caller's host arrays at the end
    uint64_t *d_hits = nullptr;  // [count][idx cap][val cap]
    Epilogue epi{};
    if (th) {
        const size_t hb_bytes = 8 * (1 + (size_t)th->cap) + esz * (size_t)th->cap;
        e = hipMalloc(&d_hits, hb_bytes);
        if (e != hipSuccess) return fail(FWHT_E_NOMEM, "streamed path: hit buffers: %s", hipGetErrorString(e));
        e = hipMemsetAsync(d_hits, 0, 8, S.scomp);
        if (e != hipSuccess) {
            (void)hipFree(d_hits);
            return hip_fail(e, "streamed path: clear count");
        }
        epi.thresh = 1;
        epi.T = th->T;
        epi.count = d_hits;
        epi.idx = d_hits + 1;
        epi.val = d_hits + 1 + th->cap;
        epi.cap = th->cap;
    }

    int lib_rc = FWHT_OK;
    uint64_t it = 0;
    // ---- row phase: low L bits of every row
    const uint64_t nrows = 1ull << H;
    for (uint64_t r0 = 0; r0 < nrows && e == hipSuccess && !lib_rc; r0 += rows_per, ++it) {
        char *src = hb + (r0 << L) * esz;
        const size_t bytes = (size_t)(rows_per << L) * esz;
        e = step(
            S, it, [&](void *d) { return hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, S.sin); },
            [&](void *d) {
                lib_rc = run_passes(d, dtype, L, rows_per, Epilogue{}, S.scomp);
                return lib_rc ? hipErrorUnknown : hipSuccess;
            },
            [&](void *d) { return hipMemcpyAsync(src, d, bytes, hipMemcpyDeviceToHost, S.sout); });
    }
    // every row must be back in host memory before any column is read
    if (e == hipSuccess && !lib_rc) e = hipStreamSynchronize(S.sout);
    // ---- column phase: high H bits of every column, threshold fused
    int wbits = 0;
    while ((1ull << wbits) < w) ++wbits;
    const uint64_t ncols = 1ull << L;
    for (uint64_t c0 = 0; c0 < ncols && e == hipSuccess && !lib_rc; c0 += w, ++it) {
        char *src = hb + c0 * esz;
        Epilogue ce = epi;
        ce.kshift = (uint32_t)wbits;
        ce.kL = (uint32_t)L;
        ce.kbase = c0;
        e = step(
            S, it,
            [&](void *d) {
                return hipMemcpy2DAsync(d, w * esz, src, ncols * esz, w * esz, nrows, hipMemcpyHostToDevice, S.sin);
            },
            [&](void *d) {
                lib_rc = run_strided_range(d, dtype, chunk, wbits, H, ce, S.scomp);
                return lib_rc ? hipErrorUnknown : hipSuccess;
            },
            [&](void *d) {
                return hipMemcpy2DAsync(src, ncols * esz, d, w * esz, w * esz, nrows, hipMemcpyDeviceToHost, S.sout);
            });
    }
    hipError_t e2 = hipStreamSynchronize(S.sin);
    hipError_t e3 = hipStreamSynchronize(S.scomp);
    hipError_t e4 = hipStreamSynchronize(S.sout);
    int ret = FWHT_OK;
    if (lib_rc) ret = lib_rc;
    else if (e != hipSuccess) ret = hip_fail(e, "streamed path");
    else if (e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess)
        ret = hip_fail(e2 != hipSuccess ? e2 : e3 != hipSuccess ? e3 : e4, "streamed path: sync");
    if (th && ret == FWHT_OK) {
        uint64_t cnt = 0;
        e = hipMemcpy(&cnt, d_hits, 8, hipMemcpyDeviceToHost);
        const uint64_t k = cnt < th->cap ? cnt : th->cap;
        if (e == hipSuccess && k) e = hipMemcpy(th->idx, d_hits + 1, 8 * k, hipMemcpyDeviceToHost);
        if (e == hipSuccess && k) e = hipMemcpy(th->val, d_hits + 1 + th->cap, esz * k, hipMemcpyDeviceToHost);
        if (e != hipSuccess) ret = hip_fail(e, "streamed path: hit copy");
        else {
            *th->count = cnt;
            if (cnt > th->cap) ret = fail(FWHT_E_CAPACITY, "%llu hits, capacity %llu", (unsigned long long)cnt,
                                          (unsigned long long)th->cap);
        }
    }
    if (d_hits) (void)hipFree(d_hits);
    return ret;
}

}  // namespace fwht
