// Temporary: entry points not built yet.
#include "fwht_internal.hpp"
namespace fwht {
int streamed_int(void *, int, int, const fwht_thresh_t *, hipStream_t) { return fail(FWHT_E_UNSUPPORTED, "streamed path not built"); }
}
