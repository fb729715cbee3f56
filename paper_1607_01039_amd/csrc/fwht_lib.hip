// fwht_lib.hip -- C ABI, pass planner and kernel registry of the gfx950 WHT
// library.  Arguments are validated on the host before anything is enqueued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fwht.h"
#include "fwht_internal.hpp"
#include "wht_tile.hpp"

namespace fwht {

// -------------------------------------------------------------- error state
static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(FWHT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------- kernel registry
// The variants of each element type are compiled in their own translation
// unit (fwht_variants_*.hip).
const std::vector<Variant> &registry(int dtype)
{
    static const std::vector<Variant> r32 = variants_u32();
    static const std::vector<Variant> r64 = variants_u64();
    static const std::vector<Variant> rf = variants_f32();
    return dtype == FWHT_I32 ? r32 : dtype == FWHT_I64 ? r64 : rf;
}

static const Variant *find_variant(int dtype, const std::string &name)
{
    for (const Variant &v : registry(dtype))
        if (name == v.name) return &v;
    return nullptr;
}

// ------------------------------------------------------------------ planner
// A schedule is a list of (variant, bits).  The first pass must be a
// contiguous variant; each later pass is strided and starts at the bit where
// the previous one stopped (its row stride is 2^b with b >= CB).
static std::mutex g_sched_mu;
static std::map<std::pair<int, int>, std::string> g_sched_override;

// A strided tile pass keeps each lane's offset from the wave's row-segment
// base in 32 bits (bytes).  In a layout that reaches global memory (the load
// layout, and every layout the pass may store from) the lane bits can include
// row bits, each worth 2^b entries, so at a large row stride b that offset
// no longer fits: such (variant, b) pairs are refused.  The register-resident
// kernels keep 64-bit lane offsets, and contiguous passes have b = CB.
static bool lane_offsets_fit(const Variant &v, int b, int dtype)
{
    if (v.whole || v.cols) return true;
    const uint32_t esz = dtype == FWHT_I64 ? 8u : 4u;
    const int K = clog2((1u << v.TB) / (uint32_t)v.NT), VB = clog2(16u / esz);
    const LayoutList L = make_layouts(v.TB, v.CB, K, VB, false);
    const int slb = std::min(8 - clog2(esz), v.CB);
    for (int p = 0; p < L.n; ++p) {
        if (p > 0 && !lanes_contiguous(L.m[p], slb)) continue;
        const uint32_t lane = low_set_bits(lowmask(v.TB) & ~L.m[p], 6);
        const uint64_t top = (((uint64_t)(lane >> v.CB)) << b) + (lane & lowmask(v.CB));
        if (top * esz >= (1ull << 32)) return false;
    }
    return true;
}

bool parse_schedule(int dtype, int n, const std::string &spec, std::vector<Pass> &out, std::string &why)
{
    out.clear();
    int done = 0;
    size_t pos = 0;
    while (pos <= spec.size() && done < n) {
        size_t e = spec.find(',', pos);
        std::string tok = spec.substr(pos, e == std::string::npos ? std::string::npos : e - pos);
        pos = e == std::string::npos ? spec.size() + 1 : e + 1;
        if (tok.empty()) continue;
        int want = -1;
        size_t c = tok.find(':');
        if (c != std::string::npos) {
            want = atoi(tok.c_str() + c + 1);
            tok = tok.substr(0, c);
        }
        const Variant *v = find_variant(dtype, tok);
        if (!v) { why = "unknown variant '" + tok + "'"; return false; }
        const int cap = v->cols ? v->TB : v->TB - v->CB;
        if (out.empty() != v->cols) { why = "first pass must be contiguous, later ones strided"; return false; }
        if (!v->cols && done < v->CB) { why = "strided pass needs b >= CB"; return false; }
        int r = want < 0 ? cap : want;
        if (r < 1 || r > cap) { why = "bit count out of range for " + tok; return false; }
        if (r > n - done) r = n - done;
        // register-resident tiles transform every bit they own: the
        // contiguous ones carry no epilogue, so strided passes must follow
        // them, and the strided ones take exactly their full height
        if (v->whole && v->cols && (r != v->TB || done + r >= n)) {
            why = "C15p/C16 cover exactly their bits and must be followed by strided passes";
            return false;
        }
        if (v->whole && !v->cols && r != cap) {
            why = "a register-resident strided variant covers exactly its full height";
            return false;
        }
        if (!lane_offsets_fit(*v, done, dtype)) {
            why = tok + " at bit " + std::to_string(done) + ": lane offsets of its row stride exceed 32 bits";
            return false;
        }
        out.push_back(Pass{v, done, r});
        done += r;
    }
    if (done < n) { why = "schedule covers fewer than n bits"; return false; }
    return true;
}

// Default schedule: the table written by the autotuner (tune/gfx950.txt next
// to the library, or $FWHT_TUNE_TABLE) when it has (dtype, n); otherwise the
// fewest passes: one contiguous pass of up to 2^15 (int64: 2^13) entries,
// then strided passes of at most 9 bits, balanced, each with a variant whose
// tile height equals its bit count and whose row segments are the widest
// (up to 1 KiB) that fit the tile.
std::string default_schedule(int dtype, int n)
{
    const std::string *tuned = tuned_schedule(dtype, n);
    if (tuned) return *tuned;
    const bool wide = dtype == FWHT_I64;
    const int cmax = wide ? 13 : 15;
    const int rmax = 9;
    // Widest row segment (up to 1 KiB) whose tile of 2^(cb + r) entries
    // still fits the 128 KiB tile limit: wide segments keep strided passes
    // close to contiguous ones in HBM efficiency.
    const int tbmax = wide ? 14 : 15, cbmax = wide ? 7 : 8;
    if (n <= 12) return wide && n <= 11 ? "C11" : "C12";
    if (n <= cmax) return "C" + std::to_string(n);
    int P = 1;
    while (cmax + rmax * (P - 1) < n) ++P;
    const int ns = P - 1;
    // Keep every strided pass at >= 3 bits (very short tiles waste lanes).
    int c = cmax;
    if (n - c < 3 * ns) c = n - 3 * ns;
    const int s = n - c;
    std::string out = "C" + std::to_string(c);
    for (int i = 0; i < ns; ++i) {
        const int r = s / ns + (i < s % ns ? 1 : 0);
        const int cb = tbmax - r < cbmax ? tbmax - r : cbmax;
        out += ",S" + std::to_string(cb + r) + "c" + std::to_string(cb) + ":" + std::to_string(r);
    }
    return out;
}

std::string schedule_for(int dtype, int n)
{
    {
        std::lock_guard<std::mutex> lk(g_sched_mu);
        auto it = g_sched_override.find({dtype, n});
        if (it != g_sched_override.end()) return it->second;
    }
    return default_schedule(dtype, n);
}

// ------------------------------------------------------------------ tracing
// When enabled, run_passes records a HIP event on the launch stream before
// the first pass and after every pass, so that the per-pass device time of
// the most recent call can be read back (the T_CPU / T_IO split of
// section 4.1, here one entry per HBM pass).
static std::mutex g_trace_mu;
static bool g_trace_on = false;
static std::vector<hipEvent_t> g_trace_ev;
static std::vector<std::string> g_trace_names;
static int g_trace_used = 0;

static hipError_t trace_record(int i, hipStream_t s)
{
    while ((int)g_trace_ev.size() <= i) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        g_trace_ev.push_back(e);
    }
    return hipEventRecord(g_trace_ev[i], s);
}

// Enqueue the passes of a transform of `batch` x 2^n entries.
int run_passes(void *buf, int dtype, int n, uint64_t batch, const Epilogue &epi, hipStream_t s, const void *src)
{
    if (n == 0) return FWHT_OK;
    std::vector<Pass> passes;
    std::string why;
    const std::string spec = schedule_for(dtype, n);
    if (!parse_schedule(dtype, n, spec, passes, why))
        return fail(FWHT_E_INVAL, "bad schedule '%s' for n=%d: %s", spec.c_str(), n, why.c_str());
    const uint64_t total = batch << n;
    std::unique_lock<std::mutex> tlk(g_trace_mu);
    const bool tr = g_trace_on;
    if (!tr) tlk.unlock();
    if (tr) {
        g_trace_names.clear();
        g_trace_used = 0;
        hipError_t e = trace_record(0, s);
        if (e != hipSuccess) return hip_fail(e, "trace event");
    }
    for (size_t p = 0; p < passes.size(); ++p) {
        const Pass &ps = passes[p];
        const Variant &v = *ps.v;
        PassArgs a{};
        a.total = total;
        if (v.cols) {
            a.b = v.CB;
            a.colblocks = 1;
            a.act = lowmask(ps.r);
            a.ntiles = (total + (1ull << v.TB) - 1) >> v.TB;
        } else {
            a.b = ps.lo;
            a.colblocks = 1ull << (ps.lo - v.CB);
            a.act = lowmask(ps.r) << v.CB;
            const uint64_t rows = total >> ps.lo;
            const int R = v.TB - v.CB;
            a.ntiles = ((rows + (1ull << R) - 1) >> R) * a.colblocks;
        }
        const bool last = p + 1 == passes.size();
        // the hit counter is cleared by the first of several passes (stream
        // order puts that before the last pass's appends); a single pass
        // needs a launch of its own for it
        if (epi.thresh && epi.clear_count) {
            if (p == 0 && !last) a.zero_first = (unsigned long long *)epi.count;
            if (p == 0 && last) {
                const int rc = zero_count(epi.count, s);
                if (rc) return rc;
            }
        }
        if (last) {
            a.kshift = epi.kshift;
            a.kL = epi.kL;
            a.kbase = epi.kbase;
            a.do_scale = epi.do_scale;
            a.scale = epi.scale;
            a.thresh = epi.thresh;
            a.T = epi.T;
            a.Tf = epi.Tf;
            a.hit_idx = (unsigned long long *)epi.idx;
            a.hit_val = epi.val;
            a.cap = epi.cap;
            a.count = (unsigned long long *)epi.count;
        }
        void *from = buf;
        if (p == 0 && src) {
            from = const_cast<void *>(src);  // read only by the kernel
            a.dst = buf;
        }
        hipError_t e = v.launch(from, a, s);
        if (e != hipSuccess) return hip_fail(e, "pass launch");
        if (tr) {
            e = trace_record((int)p + 1, s);
            if (e != hipSuccess) return hip_fail(e, "trace event");
            g_trace_names.push_back(std::string(v.name) + ":" + std::to_string(ps.lo) + "+" + std::to_string(ps.r));
            g_trace_used = (int)p + 2;
        }
    }
    return FWHT_OK;
}

// Transform bits [lo, lo + nbits) of `total` entries (a multiple of
// 2^(lo + nbits)) with strided passes only: balanced passes of at most 9 bits,
// each on the variant whose tile height equals its bit count, over 256-byte
// row segments (512-byte when a pass takes a single bit).  The epilogue goes
// on the last pass.
int run_strided_range(void *buf, int dtype, uint64_t total, int lo, int nbits, const Epilogue &epi, hipStream_t s)
{
    if (nbits <= 0) return FWHT_OK;
    const int tbmax = dtype == FWHT_I64 ? 14 : 15, cbmax = dtype == FWHT_I64 ? 7 : 8;
    const int np = (nbits + 8) / 9;
    // every pass is chosen and checked before the first one is launched
    std::vector<Pass> passes;
    for (int i = 0, done = lo; i < np; ++i) {
        const int r = nbits / np + (i < nbits % np ? 1 : 0);
        // the widest row segment that fits the tile and lies below bit `done`
        int c = tbmax - r < cbmax ? tbmax - r : cbmax;
        if (c > done) c = done;
        const Variant *v = nullptr;
        for (; c >= 4 && !v; --c) v = find_variant(dtype, "S" + std::to_string(c + r) + "c" + std::to_string(c));
        if (!v) return fail(FWHT_E_UNSUPPORTED, "no strided variant for %d bits at bit %d", r, done);
        if (done < v->CB) return fail(FWHT_E_INVAL, "strided range starts below the row segment");
        if (!lane_offsets_fit(*v, done, dtype))
            return fail(FWHT_E_UNSUPPORTED, "%s at bit %d: lane offsets exceed 32 bits", v->name, done);
        passes.push_back(Pass{v, done, r});
        done += r;
    }
    for (int i = 0; i < np; ++i) {
        const Variant *v = passes[i].v;
        const int done = passes[i].lo, r = passes[i].r;
        PassArgs a{};
        a.total = total;
        a.b = done;
        a.colblocks = 1ull << (done - v->CB);
        a.act = lowmask(r) << v->CB;
        const uint64_t rows = total >> done;
        a.ntiles = ((rows + (1ull << (v->TB - v->CB)) - 1) >> (v->TB - v->CB)) * a.colblocks;
        if (i + 1 == np) {
            a.kshift = epi.kshift;
            a.kL = epi.kL;
            a.kbase = epi.kbase;
            a.do_scale = epi.do_scale;
            a.scale = epi.scale;
            a.thresh = epi.thresh;
            a.T = epi.T;
            a.Tf = epi.Tf;
            a.hit_idx = (unsigned long long *)epi.idx;
            a.hit_val = epi.val;
            a.cap = epi.cap;
            a.count = (unsigned long long *)epi.count;
        }
        hipError_t e = v->launch(buf, a, s);
        if (e != hipSuccess) return hip_fail(e, "strided pass launch");
    }
    return FWHT_OK;
}

// ------------------------------------------------------------ small kernels
__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0ull; }

int zero_count(uint64_t *count, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, (unsigned long long *)count);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FWHT_OK : hip_fail(e, "zero count");
}

// Stand-alone threshold pass: each workgroup takes blocks of 4 x 256
// 16-byte vectors (a wave's load covers 64 consecutive vectors), issues the
// four loads before testing any of them, and tests a whole block with one
// add and compare per entry OR-ed into a lane flag; only a wave with a hit
// appends, per entry, through the wave-aggregated emission.
template <class S>
__global__ void __launch_bounds__(256) threshold_kernel(const S *__restrict__ y, uint64_t len, PassArgs a)
{
    constexpr int VEC = 16 / sizeof(S), U = 4;
    const HitTest<S> ht(a);
    const uint32_t t = threadIdx.x;
    for (uint64_t blk = blockIdx.x;; blk += gridDim.x) {
        const uint64_t e0 = blk * (256u * U * VEC);  // first entry of the block
        if (e0 >= len) break;
        if (e0 + 256u * U * VEC <= len) {
            uint4 q[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                q[u] = *reinterpret_cast<const uint4 *>(y + e0 + ((uint64_t)u * 256u + t) * VEC);
            bool any = false;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const S *qs = reinterpret_cast<const S *>(&q[u]);
#pragma unroll
                for (int e = 0; e < VEC; ++e) any |= ht.above(qs[e]);
            }
            if (__ballot(any) == 0) continue;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const S *qs = reinterpret_cast<const S *>(&q[u]);
                const uint64_t k0 = e0 + ((uint64_t)u * 256u + t) * VEC;
#pragma unroll
                for (int e = 0; e < VEC; ++e) emit_hits<S>(ht.above(qs[e]), k0 + e, qs[e], a);
            }
        } else {
            // the last, partial block: entry by entry with bounds
            for (int u = 0; u < U; ++u) {
                const uint64_t k0 = e0 + ((uint64_t)u * 256u + t) * VEC;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const bool in = k0 + e < len;
                    const S x = in ? y[k0 + e] : S(0);
                    emit_hits<S>(in && ht.above(x), k0 + e, x, a);
                }
            }
        }
    }
}

__global__ void __launch_bounds__(256) copy_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src, uint64_t n16)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * 256)
        dst[i] = src[i];
}

float float_threshold(double T)
{
    // Largest float <= T: |y| > T  <=>  |y| > Tf for every float y.
    if (std::isnan(T)) return NAN;
    if (T >= 3.4028234663852886e38) return INFINITY;
    if (T < -3.4028234663852886e38) return -INFINITY;
    float f = (float)T;
    if ((double)f > T) f = std::nextafter(f, -INFINITY);
    return f;
}

bool is_device_pointer(const void *p, bool *is_host_pinned)
{
    hipPointerAttribute_t at;
    *is_host_pinned = false;
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (at.type == hipMemoryTypeHost) { *is_host_pinned = true; return false; }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

}  // namespace fwht

using namespace fwht;

// ====================================================================== C ABI
extern "C" {

const char *fwht_last_error(void) { return g_err.c_str(); }

const char *fwht_version(void) { return "fwht-gfx950 0.1"; }

static int check_thresh(const fwht_thresh_t *th)
{
    if (!th) return FWHT_OK;
    if (!th->count) return fail(FWHT_E_INVAL, "threshold: count is NULL");
    if (th->cap > 0 && (!th->idx || !th->val)) return fail(FWHT_E_INVAL, "threshold: idx/val NULL with cap > 0");
    return FWHT_OK;
}

int fwht_int(void *data, int dtype, int n, const fwht_thresh_t *th, void *stream)
{
    g_err.clear();
    if (!data) return fail(FWHT_E_INVAL, "data is NULL");
    if (((uintptr_t)data) & 15) return fail(FWHT_E_INVAL, "data must be 16-byte aligned");
    if (dtype != FWHT_I32 && dtype != FWHT_I64) return fail(FWHT_E_INVAL, "dtype must be FWHT_I32 or FWHT_I64");
    if (n < 0) return fail(FWHT_E_RANGE, "n must be >= 0");
    if (dtype == FWHT_I32 && n > 30) return fail(FWHT_E_RANGE, "int32 transforms are limited to n <= 30");
    int rc = check_thresh(th);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    bool pinned = false;
    const bool dev = is_device_pointer(data, &pinned);
    if (!dev) {
        if (!pinned) return fail(FWHT_E_INVAL, "data is neither device nor pinned host memory");
        if (th && th->cap > 0 && (!th->idx || !th->val)) return fail(FWHT_E_INVAL, "threshold: idx/val NULL");
        return streamed_int(data, dtype, n, th, s);
    }
    // 2^35 int64 entries (256 GiB) still fit one GPU's 288 GB of HBM
    if (n > 35) return fail(FWHT_E_RANGE, "in-HBM transforms are limited to n <= 35");
    Epilogue epi{};
    if (th) {
        epi.thresh = 1;
        epi.T = th->T;
        epi.idx = th->idx;
        epi.val = th->val;
        epi.cap = th->cap;
        epi.count = th->count;
        epi.clear_count = 1;
        if (n == 0) return fwht_threshold(data, dtype, 0, th, stream);
    }
    return run_passes(data, dtype, n, 1, epi, s);
}

int fwht_float(float *data, int n, int64_t batch, int normalize, int prec, void *stream)
{
    g_err.clear();
    if (!data) return fail(FWHT_E_INVAL, "data is NULL");
    if (((uintptr_t)data) & 15) return fail(FWHT_E_INVAL, "data must be 16-byte aligned");
    if (n < 0 || n > 30) return fail(FWHT_E_RANGE, "fwht_float needs 0 <= n <= 30");
    if (batch < 1) return fail(FWHT_E_INVAL, "batch must be >= 1");
    if (n + 64 - __builtin_clzll((unsigned long long)batch) > 40) return fail(FWHT_E_RANGE, "batch * 2^n too large");
    if (prec != FWHT_PREC_FP32 && prec != FWHT_PREC_FP16_MFMA && prec != FWHT_PREC_BF16_MFMA)
        return fail(FWHT_E_INVAL, "unknown precision %d", prec);
    hipStream_t s = (hipStream_t)stream;
    if (prec != FWHT_PREC_FP32) return mfma_uniform(data, n, (uint64_t)batch, normalize, prec, s);
    Epilogue epi{};
    if (normalize && n > 0) {
        epi.do_scale = 1;
        epi.scale = (float)(1.0 / std::sqrt(std::ldexp(1.0, n)));
    }
    return run_passes(data, FWHT_F32, n, (uint64_t)batch, epi, s);
}

int fwht_float_out(const float *src, float *dst, int n, int64_t batch, int normalize, int prec, void *stream)
{
    g_err.clear();
    if (!src || !dst) return fail(FWHT_E_INVAL, "src or dst is NULL");
    if ((((uintptr_t)src) | ((uintptr_t)dst)) & 15) return fail(FWHT_E_INVAL, "src and dst must be 16-byte aligned");
    if (n < 0 || n > 30) return fail(FWHT_E_RANGE, "fwht_float_out needs 0 <= n <= 30");
    if (batch < 1) return fail(FWHT_E_INVAL, "batch must be >= 1");
    if (n + 64 - __builtin_clzll((unsigned long long)batch) > 40) return fail(FWHT_E_RANGE, "batch * 2^n too large");
    if (prec != FWHT_PREC_FP32 && prec != FWHT_PREC_FP16_MFMA && prec != FWHT_PREC_BF16_MFMA)
        return fail(FWHT_E_INVAL, "unknown precision %d", prec);
    if (src == dst) return fwht_float(dst, n, batch, normalize, prec, stream);
    const uint64_t bytes = ((uint64_t)batch << n) * sizeof(float);
    const uintptr_t a0 = (uintptr_t)src, b0 = (uintptr_t)dst;
    if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(FWHT_E_INVAL, "src and dst overlap");
    hipStream_t s = (hipStream_t)stream;
    if (prec != FWHT_PREC_FP32 || n == 0) {
        // the matrix-core kernels work in place: copy, then transform dst
        // (their limits checked first, so that a refused call enqueues nothing)
        if (prec != FWHT_PREC_FP32 && (n < 4 || n > 16))
            return fail(FWHT_E_UNSUPPORTED, "MFMA precisions need 4 <= n <= 16 (got %d)", n);
        if (prec != FWHT_PREC_FP32 && (uint64_t)batch > (uint64_t)0x7fffffff)
            return fail(FWHT_E_RANGE, "batch too large for the MFMA path");
        const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "copy src to dst");
        return fwht_float(dst, n, batch, normalize, prec, stream);
    }
    Epilogue epi{};
    if (normalize) {
        epi.do_scale = 1;
        epi.scale = (float)(1.0 / std::sqrt(std::ldexp(1.0, n)));
    }
    return run_passes(dst, FWHT_F32, n, (uint64_t)batch, epi, s, src);
}

int fwht_threshold(const void *data, int dtype, int n, const fwht_thresh_t *th, void *stream)
{
    if (!data) return fail(FWHT_E_INVAL, "data is NULL");
    if (((uintptr_t)data) & 15) return fail(FWHT_E_INVAL, "data must be 16-byte aligned");
    if (dtype != FWHT_I32 && dtype != FWHT_I64 && dtype != FWHT_F32) return fail(FWHT_E_INVAL, "bad dtype");
    if (n < 0 || n > 40) return fail(FWHT_E_RANGE, "n out of range");
    if (!th) return fail(FWHT_E_INVAL, "threshold request is NULL");
    int rc = check_thresh(th);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = zero_count(th->count, s);
    if (rc) return rc;
    PassArgs a{};
    a.thresh = 1;
    a.T = th->T;
    a.Tf = float_threshold(th->Tf);
    a.hit_idx = (unsigned long long *)th->idx;
    a.hit_val = th->val;
    a.cap = th->cap;
    a.count = (unsigned long long *)th->count;
    const uint64_t len = 1ull << n;
    const int esz = dtype == FWHT_I64 ? 8 : 4;
    const uint64_t vecs = (len * esz + 15) / 16;
    uint64_t grid = (vecs + 4 * 256 - 1) / (4 * 256);  // blocks of 4 x 256 vectors
    if (grid > 256 * 16) grid = 256 * 16;
    if (dtype == FWHT_I32)
        hipLaunchKernelGGL(threshold_kernel<uint32_t>, dim3((uint32_t)grid), dim3(256), 0, s, (const uint32_t *)data, len, a);
    else if (dtype == FWHT_I64)
        hipLaunchKernelGGL(threshold_kernel<uint64_t>, dim3((uint32_t)grid), dim3(256), 0, s, (const uint64_t *)data, len, a);
    else
        hipLaunchKernelGGL(threshold_kernel<float>, dim3((uint32_t)grid), dim3(256), 0, s, (const float *)data, len, a);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FWHT_OK : hip_fail(e, "threshold launch");
}

int fwht_set_schedule(int dtype, int n, const char *spec)
{
    g_err.clear();
    if (dtype != FWHT_I32 && dtype != FWHT_I64 && dtype != FWHT_F32) return fail(FWHT_E_INVAL, "bad dtype");
    if (n < 1 || n > 40) return fail(FWHT_E_RANGE, "n out of range");
    std::lock_guard<std::mutex> lk(g_sched_mu);
    if (!spec) {
        g_sched_override.erase({dtype, n});
        return FWHT_OK;
    }
    std::vector<Pass> p;
    std::string why;
    if (!parse_schedule(dtype, n, spec, p, why)) return fail(FWHT_E_INVAL, "schedule '%s': %s", spec, why.c_str());
    g_sched_override[{dtype, n}] = spec;
    return FWHT_OK;
}

int fwht_list_variants(int dtype, char *buf, int len)
{
    if (!buf || len < 1) return fail(FWHT_E_INVAL, "bad buffer");
    if (dtype != FWHT_I32 && dtype != FWHT_I64 && dtype != FWHT_F32) return fail(FWHT_E_INVAL, "bad dtype");
    std::string all;
    for (const Variant &v : registry(dtype)) {
        if (!all.empty()) all += ",";
        all += v.name;
    }
    snprintf(buf, (size_t)len, "%s", all.c_str());
    return FWHT_OK;
}

int fwht_get_schedule(int dtype, int n, char *buf, int len)
{
    if (!buf || len < 1) return fail(FWHT_E_INVAL, "bad buffer");
    std::string s = schedule_for(dtype, n);
    snprintf(buf, (size_t)len, "%s", s.c_str());
    return FWHT_OK;
}

int fwht_trace_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_trace_mu);
    g_trace_on = on != 0;
    g_trace_used = 0;
    return FWHT_OK;
}

int fwht_trace_read(float *ms, int cap, int *count, char *names, int names_len)
{
    std::lock_guard<std::mutex> lk(g_trace_mu);
    if (!count) return fail(FWHT_E_INVAL, "count is NULL");
    const int np = g_trace_used > 0 ? g_trace_used - 1 : 0;
    *count = np;
    if (np == 0) return FWHT_OK;
    hipError_t e = hipEventSynchronize(g_trace_ev[np]);
    if (e != hipSuccess) return hip_fail(e, "trace sync");
    std::string all;
    for (int i = 0; i < np; ++i) {
        float t = 0.f;
        e = hipEventElapsedTime(&t, g_trace_ev[i], g_trace_ev[i + 1]);
        if (e != hipSuccess) return hip_fail(e, "trace elapsed");
        if (ms && i < cap) ms[i] = t;
        if (i) all += ",";
        all += g_trace_names[i];
    }
    if (names && names_len > 0) snprintf(names, (size_t)names_len, "%s", all.c_str());
    return FWHT_OK;
}

int fwht_copy(void *dst, const void *src, uint64_t bytes, void *stream)
{
    if (!dst || !src || (((uintptr_t)dst | (uintptr_t)src | bytes) & 15))
        return fail(FWHT_E_INVAL, "copy needs 16-byte aligned pointers and size");
    const uint64_t n16 = bytes / 16;
    // one 16-byte vector per thread while the grid allows (measured the
    // fastest streaming copy on this GPU: 6.2 TB/s against 4.8 with a
    // grid-stride loop over a capped grid); the dispatch counts work-items
    // in 32 bits, so beyond 2^31 vectors the kernel loops
    uint64_t grid = (n16 + 255) / 256;
    if (grid > (1ull << 31) / 256) grid = (1ull << 31) / 256;
    if (grid == 0) return FWHT_OK;
    hipLaunchKernelGGL(copy_kernel, dim3((uint32_t)grid), dim3(256), 0, (hipStream_t)stream,
                       (uint4 *)dst, (const uint4 *)src, n16);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FWHT_OK : hip_fail(e, "copy launch");
}

}  // extern "C"
