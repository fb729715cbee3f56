// Temporary: entry points not built yet.
#include "fwht_internal.hpp"
namespace fwht {
int streamed_int(void *, int, int, const fwht_thresh_t *, hipStream_t) { return fail(FWHT_E_UNSUPPORTED, "streamed path not built"); }
int mfma_uniform(float *, int, uint64_t, int, int, hipStream_t) { return fail(FWHT_E_UNSUPPORTED, "mfma path not built"); }
}
extern "C" {
int fwht_batched(float *, const int64_t *, const int32_t *, int32_t, int, int, void *) { return fwht::fail(FWHT_E_UNSUPPORTED, "batched not built"); }
int fwht_norms(const float *, const float *, const double *, const int64_t *, const int32_t *, int32_t, double *, void *) { return fwht::fail(FWHT_E_UNSUPPORTED, "norms not built"); }
}
