// Temporary: entry points not built yet.
#include "fwht_internal.hpp"
namespace fwht {
int streamed_int(void *, int, int, const fwht_thresh_t *, hipStream_t) { return fail(FWHT_E_UNSUPPORTED, "streamed path not built"); }
int mfma_uniform(float *, int, uint64_t, int, int, hipStream_t) { return fail(FWHT_E_UNSUPPORTED, "mfma path not built"); }
hipError_t launch_batched_mfma(int, const BArgs &, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t batched_mfma_occupancy(int, int *b) { *b = 1; return hipSuccess; }
}
