// Matrix-core (MFMA) kernels for the large float32 per-slice products.
#include "common.hpp"

namespace tp {

int cgemm_mfma(const CGemm&, int, hipStream_t, bool* handled) {
  *handled = false;
  return TP_OK;
}

}  // namespace tp
