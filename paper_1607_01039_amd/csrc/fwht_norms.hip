// fwht_norms.hip -- FP64 per-transform sums of squares (section 2: the
// orthonormal transform keeps the sum of squares, so sum y^2 = sum x^2 up to
// rounding; with a reference r, sum (y - r)^2 gives the error norm).  These
// reductions are the only FP64 arithmetic on the GPU.
#include <hip/hip_runtime.h>

#include <vector>

#include "fwht_internal.hpp"

namespace fwht {

struct NormItem {
    int64_t off;
    int64_t len;
};

__global__ void __launch_bounds__(256) norms_kernel(const float *__restrict__ x, const float *__restrict__ y,
                                                    const double *__restrict__ r, const NormItem *__restrict__ items,
                                                    double *__restrict__ out)
{
    __shared__ double red[3][256];
    const NormItem it = items[blockIdx.x];
    double sx = 0.0, sy = 0.0, se = 0.0;
    for (int64_t i = threadIdx.x; i < it.len; i += 256) {
        const double xv = x[it.off + i], yv = y[it.off + i];
        sx += xv * xv;
        sy += yv * yv;
        if (r) {
            const double d = yv - r[it.off + i];
            se += d * d;
        }
    }
    red[0][threadIdx.x] = sx;
    red[1][threadIdx.x] = sy;
    red[2][threadIdx.x] = se;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[3 * (int64_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

int norms(const float *x, const float *y, const double *r, const int64_t *offsets, const int32_t *log2n,
          int32_t count, double *out, hipStream_t s)
{
    std::vector<NormItem> items((size_t)count);
    for (int32_t t = 0; t < count; ++t) {
        if (log2n[t] < 0 || log2n[t] > 30) return fail(FWHT_E_RANGE, "log2n[%d] = %d out of range", t, log2n[t]);
        if (offsets[t] < 0) return fail(FWHT_E_INVAL, "offsets[%d] < 0", t);
        items[(size_t)t] = NormItem{offsets[t], (int64_t)1 << log2n[t]};
    }
    // Per-call metadata in stream-ordered memory: allocated, filled, read and
    // released in the order of `s`, so concurrent calls never share it.
    const size_t bytes = sizeof(NormItem) * (size_t)count;
    void *d_items = nullptr;
    hipError_t e = hipMallocAsync(&d_items, bytes, s);
    if (e != hipSuccess) return fail(FWHT_E_NOMEM, "norms: %s", hipGetErrorString(e));
    e = hipMemcpyAsync(d_items, items.data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // `items` is pageable and local
    if (e != hipSuccess) {
        (void)hipFreeAsync(d_items, s);
        return hip_fail(e, "norms upload");
    }
    hipLaunchKernelGGL(norms_kernel, dim3((uint32_t)count), dim3(256), 0, s, x, y, r, (const NormItem *)d_items,
                       out);
    e = hipGetLastError();
    (void)hipFreeAsync(d_items, s);
    return e == hipSuccess ? FWHT_OK : hip_fail(e, "norms launch");
}

}  // namespace fwht

extern "C" int fwht_norms(const float *x, const float *y, const double *r, const int64_t *offsets,
                          const int32_t *log2n, int32_t count, double *out, void *stream)
{
    if (!x || !y || !offsets || !log2n || !out) return fwht::fail(FWHT_E_INVAL, "NULL argument");
    if (count < 1) return fwht::fail(FWHT_E_INVAL, "count must be >= 1");
    // one workgroup of 256 per transform; the dispatch counts work-items in 32 bits
    if (count > (1 << 23)) return fwht::fail(FWHT_E_RANGE, "count must be <= 2^23");
    return fwht::norms(x, y, r, offsets, log2n, count, out, (hipStream_t)stream);
}
