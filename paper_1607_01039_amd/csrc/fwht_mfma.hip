// fwht_mfma.hip -- launchers of the matrix-core (f16 / bf16 operand) batched
// kernel, and fwht_float's MFMA precisions (uniform sizes through the batched
// path).
#include <hip/hip_runtime.h>

#include <vector>

#include "fwht_internal.hpp"
#include "wht_batched_mfma.hpp"

namespace fwht {

hipError_t launch_batched_mfma(int prec, const BArgs &a, int grid, hipStream_t s)
{
    if (prec == FWHT_PREC_FP16_MFMA)
        hipLaunchKernelGGL(batched_mfma_kernel<FWHT_PREC_FP16_MFMA>, dim3(grid), dim3(1024), 0, s, a);
    else if (prec == FWHT_PREC_BF16_MFMA)
        hipLaunchKernelGGL(batched_mfma_kernel<FWHT_PREC_BF16_MFMA>, dim3(grid), dim3(1024), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t batched_mfma_occupancy(int prec, int *blocks_per_cu)
{
    if (prec == FWHT_PREC_FP16_MFMA)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batched_mfma_kernel<FWHT_PREC_FP16_MFMA>,
                                                            1024, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batched_mfma_kernel<FWHT_PREC_BF16_MFMA>,
                                                        1024, 0);
}

// `batch` transforms of 2^n consecutive entries through the batched kernel.
int mfma_uniform(float *data, int n, uint64_t batch, int normalize, int prec, hipStream_t s)
{
    if (n < 4 || n > 16) return fail(FWHT_E_UNSUPPORTED, "MFMA precisions need 4 <= n <= 16 (got %d)", n);
    if (batch > (uint64_t)0x7fffffff) return fail(FWHT_E_RANGE, "batch too large for the MFMA path");
    std::vector<int64_t> off(batch);
    std::vector<int32_t> lg(batch, n);
    for (uint64_t t = 0; t < batch; ++t) off[t] = (int64_t)(t << n);
    return batched(data, off.data(), lg.data(), (int32_t)batch, normalize, prec, s);
}

}  // namespace fwht
