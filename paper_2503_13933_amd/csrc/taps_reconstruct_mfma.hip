// Reduced-precision reconstruction on the matrix cores (placeholder until the
// MFMA kernels land): reports TAPS_ERR_UNSUPPORTED.
#include "taps_internal.hpp"

namespace taps {
taps_status reconstruct_mfma(taps_handle* h, const int32_t*, const double* const*, int32_t, const double*,
                             taps_prec, taps_recon_mode, void*, double, hipStream_t) {
  return fail(h, TAPS_ERR_UNSUPPORTED, "FP32/BF16 reconstruction not built yet");
}
}  // namespace taps
