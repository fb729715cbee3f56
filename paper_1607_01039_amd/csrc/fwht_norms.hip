// fwht_norms.hip -- FP64 per-transform sums of squares (section 2: the
// orthonormal transform keeps the sum of squares, so sum y^2 = sum x^2 up to
// rounding; with a reference r, sum (y - r)^2 gives the error norm).  These
// reductions are the only FP64 arithmetic on the GPU.
//
// Two launches: every transform is cut into chunks of at most 2^12 entries,
// one workgroup reduces a chunk to three partial sums (16-byte loads when the
// chunk is aligned), and one thread per transform then adds its chunks'
// partials in chunk order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cstring>
#include <list>
#include <mutex>
#include <vector>

#include "fwht_internal.hpp"

namespace fwht {

constexpr int kNormThreads = 256;
constexpr int kNormChunkBits = 12;
constexpr uint32_t kNormMaxGrid = 1u << 16;  // workgroups of the partial pass; it loops over chunks

struct NormChunk {
    int64_t off;  // first entry
    int32_t len;  // entries (<= 2^12)
    int32_t pad;
};

__device__ __forceinline__ void acc(double &s, float v) { s = fma((double)v, (double)v, s); }

__global__ void __launch_bounds__(kNormThreads) norms_partial_kernel(const float *__restrict__ x,
                                                                     const float *__restrict__ y,
                                                                     const double *__restrict__ r,
                                                                     const NormChunk *__restrict__ chunks,
                                                                     uint32_t nchunks, int vec_ok,
                                                                     double *__restrict__ part)
{
    __shared__ double red[3][kNormThreads / 64];
    const uint32_t t = threadIdx.x;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const NormChunk ch = chunks[c];
        double sx = 0.0, sy = 0.0, se = 0.0;
        if (vec_ok && ((ch.off | ch.len) & 3) == 0) {
            // 16-byte loads: four entries of x and y, two 16-byte loads of r
            const float4 *x4 = reinterpret_cast<const float4 *>(x + ch.off);
            const float4 *y4 = reinterpret_cast<const float4 *>(y + ch.off);
            const double2 *r2 = r ? reinterpret_cast<const double2 *>(r + ch.off) : nullptr;
            const int32_t nv = ch.len / 4;
            int32_t i = (int32_t)t;
            // four of this thread's vectors per round, every load issued
            // before the first is used; the sums take them in the same order
            for (; i + 3 * kNormThreads < nv; i += 4 * kNormThreads) {
                float4 a[4], b[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] = x4[i + u * kNormThreads], b[u] = y4[i + u * kNormThreads];
                if (r2) {
                    double2 p[4], q[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        p[u] = r2[2 * (i + u * kNormThreads)], q[u] = r2[2 * (i + u * kNormThreads) + 1];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double d0 = (double)b[u].x - p[u].x, d1 = (double)b[u].y - p[u].y;
                        const double d2 = (double)b[u].z - q[u].x, d3 = (double)b[u].w - q[u].y;
                        se = fma(d0, d0, se), se = fma(d1, d1, se), se = fma(d2, d2, se), se = fma(d3, d3, se);
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc(sx, a[u].x), acc(sx, a[u].y), acc(sx, a[u].z), acc(sx, a[u].w);
                    acc(sy, b[u].x), acc(sy, b[u].y), acc(sy, b[u].z), acc(sy, b[u].w);
                }
            }
            for (; i < nv; i += kNormThreads) {
                const float4 a = x4[i], b = y4[i];
                acc(sx, a.x), acc(sx, a.y), acc(sx, a.z), acc(sx, a.w);
                acc(sy, b.x), acc(sy, b.y), acc(sy, b.z), acc(sy, b.w);
                if (r2) {
                    const double2 p = r2[2 * i], q = r2[2 * i + 1];
                    const double d0 = (double)b.x - p.x, d1 = (double)b.y - p.y;
                    const double d2 = (double)b.z - q.x, d3 = (double)b.w - q.y;
                    se = fma(d0, d0, se), se = fma(d1, d1, se), se = fma(d2, d2, se), se = fma(d3, d3, se);
                }
            }
        } else {
            for (int32_t i = (int32_t)t; i < ch.len; i += kNormThreads) {
                const float a = x[ch.off + i], b = y[ch.off + i];
                acc(sx, a);
                acc(sy, b);
                if (r) {
                    const double d = (double)b - r[ch.off + i];
                    se = fma(d, d, se);
                }
            }
        }
        // wave sums (lane order fixed), then the four waves in order
        for (int m = 32; m > 0; m >>= 1) {
            sx += __shfl_xor(sx, m);
            sy += __shfl_xor(sy, m);
            se += __shfl_xor(se, m);
        }
        if ((t & 63u) == 0) {
            red[0][t >> 6] = sx;
            red[1][t >> 6] = sy;
            red[2][t >> 6] = se;
        }
        __syncthreads();
        if (t < 3) {
            double s = 0.0;
            for (int w = 0; w < kNormThreads / 64; ++w) s += red[t][w];
            part[3 * (uint64_t)c + t] = s;
        }
        __syncthreads();  // red is reused by the next chunk
    }
}

// out[3t + k] = sum over the chunks of transform t (first[t] .. first[t + 1] - 1) of their partials
__global__ void __launch_bounds__(kNormThreads) norms_final_kernel(const double *__restrict__ part,
                                                                   const uint32_t *__restrict__ first,
                                                                   int32_t count, double *__restrict__ out)
{
    const int64_t tr = (int64_t)blockIdx.x * kNormThreads + threadIdx.x;
    if (tr >= count) return;
    double s[3] = {0.0, 0.0, 0.0};
    const uint32_t c1 = first[tr + 1];
    uint32_t c = first[tr];
    // four chunks' partials loaded before they are added, in chunk order
    for (; c + 4 <= c1; c += 4) {
        double q[12];
#pragma unroll
        for (int u = 0; u < 12; ++u) q[u] = part[3 * (uint64_t)c + u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            for (int k = 0; k < 3; ++k) s[k] += q[3 * u + k];
    }
    for (; c < c1; ++c)
        for (int k = 0; k < 3; ++k) s[k] += part[3 * (uint64_t)c + k];
    for (int k = 0; k < 3; ++k) out[3 * tr + k] = s[k];
}

// The chunk table of a request (the chunks, then first[count + 1]) is built
// on the host, uploaded once and kept for later calls with the same offsets
// and sizes on the same device (a few most recent requests), together with
// the buffer of partial sums that those calls share.  A call records an event
// after its last kernel and the next call of the same request, on whatever
// stream, waits for it, so no call overwrites partial sums another is still
// adding.
struct NormPlan {
    int dev = 0;
    std::vector<int64_t> off;
    std::vector<int32_t> lg;
    char *table = nullptr;  // device: NormChunk[nchunks], then uint32 first[count + 1] at foff
    double *part = nullptr;  // device: 3 partial sums per chunk
    hipEvent_t done = nullptr;  // recorded after the last call's final kernel
    bool used = false;
    uint32_t nchunks = 0;
    size_t foff = 0;
};

void release(NormPlan &p)
{
    if (p.table) (void)hipFree(p.table);
    if (p.part) (void)hipFree(p.part);
    if (p.done) (void)hipEventDestroy(p.done);
    p.table = nullptr;
    p.part = nullptr;
    p.done = nullptr;
}
std::mutex g_norm_mu;
std::list<NormPlan> g_norm_plans;  // most recent first
constexpr size_t kMaxNormPlans = 4;

int make_norm_plan(NormPlan &p, const int64_t *offsets, const int32_t *log2n, int32_t count)
{
    size_t total = 0;
    for (int32_t t = 0; t < count; ++t) {
        if (log2n[t] < 0 || log2n[t] > 30) return fail(FWHT_E_RANGE, "log2n[%d] = %d out of range", t, log2n[t]);
        if (offsets[t] < 0) return fail(FWHT_E_INVAL, "offsets[%d] < 0", t);
        total += (((size_t)1 << log2n[t]) + ((size_t)1 << kNormChunkBits) - 1) >> kNormChunkBits;
    }
    // chunk indices stay below 2^30, so the grid-stride loop never wraps
    if (total > ((size_t)1 << 30)) return fail(FWHT_E_RANGE, "too many entries for the norm reductions");
    std::vector<NormChunk> chunks;
    chunks.reserve(total);
    std::vector<uint32_t> first((size_t)count + 1);
    for (int32_t t = 0; t < count; ++t) {
        const int64_t len = (int64_t)1 << log2n[t];
        first[(size_t)t] = (uint32_t)chunks.size();
        for (int64_t c = 0; c < len; c += (int64_t)1 << kNormChunkBits) {
            const int64_t l = len - c < ((int64_t)1 << kNormChunkBits) ? len - c : ((int64_t)1 << kNormChunkBits);
            chunks.push_back(NormChunk{offsets[t] + c, (int32_t)l, 0});
        }
    }
    first[(size_t)count] = (uint32_t)chunks.size();
    p.nchunks = (uint32_t)chunks.size();
    const size_t cbytes = sizeof(NormChunk) * chunks.size(), fbytes = sizeof(uint32_t) * first.size();
    p.foff = (cbytes + 15) & ~(size_t)15;
    hipError_t e = hipMalloc((void **)&p.table, p.foff + fbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&p.part, sizeof(double) * 3 * chunks.size());
    if (e != hipSuccess) return fail(FWHT_E_NOMEM, "norms table: %s", hipGetErrorString(e));
    e = hipEventCreateWithFlags(&p.done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "norms event");
    e = hipMemcpy(p.table, chunks.data(), cbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p.table + p.foff, first.data(), fbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "norms table upload");
    p.off.assign(offsets, offsets + count);
    p.lg.assign(log2n, log2n + count);
    return FWHT_OK;
}

int norms(const float *x, const float *y, const double *r, const int64_t *offsets, const int32_t *log2n,
          int32_t count, double *out, hipStream_t s)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    std::lock_guard<std::mutex> lk(g_norm_mu);
    auto it = g_norm_plans.begin();
    for (; it != g_norm_plans.end(); ++it)
        if (it->dev == dev && it->off.size() == (size_t)count &&
            !memcmp(it->lg.data(), log2n, sizeof(int32_t) * (size_t)count) &&
            !memcmp(it->off.data(), offsets, sizeof(int64_t) * (size_t)count))
            break;
    if (it == g_norm_plans.end()) {
        NormPlan p;
        p.dev = dev;
        const int rc = make_norm_plan(p, offsets, log2n, count);
        if (rc) {
            release(p);
            return rc;
        }
        if (g_norm_plans.size() >= kMaxNormPlans) {
            // an evicted plan may still be used by work in flight on some stream
            (void)hipDeviceSynchronize();
            release(g_norm_plans.back());
            g_norm_plans.pop_back();
        }
        g_norm_plans.push_front(std::move(p));
        it = g_norm_plans.begin();
    } else if (it != g_norm_plans.begin()) {
        g_norm_plans.splice(g_norm_plans.begin(), g_norm_plans, it);
        it = g_norm_plans.begin();
    }
    NormPlan &p = *it;
    // 16-byte loads need 16-byte aligned bases (chunk offsets are checked per chunk)
    const int vec_ok = ((((uintptr_t)x) | ((uintptr_t)y) | ((uintptr_t)r)) & 15) == 0;
    if (p.used) {
        e = hipStreamWaitEvent(s, p.done, 0);
        if (e != hipSuccess) return hip_fail(e, "norms: wait for the previous call");
    }
    const uint32_t grid = p.nchunks < kNormMaxGrid ? p.nchunks : kNormMaxGrid;
    hipLaunchKernelGGL(norms_partial_kernel, dim3(grid), dim3(kNormThreads), 0, s, x, y, r,
                       (const NormChunk *)p.table, p.nchunks, vec_ok, p.part);
    e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(norms_final_kernel, dim3((uint32_t)((count + kNormThreads - 1) / kNormThreads)),
                           dim3(kNormThreads), 0, s, (const double *)p.part,
                           (const uint32_t *)(p.table + p.foff), count, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(p.done, s);
    if (e != hipSuccess) return hip_fail(e, "norms launch");
    p.used = true;
    return FWHT_OK;
}

}  // namespace fwht

extern "C" int fwht_norms(const float *x, const float *y, const double *r, const int64_t *offsets,
                          const int32_t *log2n, int32_t count, double *out, void *stream)
{
    if (!x || !y || !offsets || !log2n || !out) return fwht::fail(FWHT_E_INVAL, "NULL argument");
    if (count < 1) return fwht::fail(FWHT_E_INVAL, "count must be >= 1");
    if (count > (1 << 23)) return fwht::fail(FWHT_E_RANGE, "count must be <= 2^23");
    return fwht::norms(x, y, r, offsets, log2n, count, out, (hipStream_t)stream);
}
