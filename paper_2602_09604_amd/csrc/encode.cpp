// Device encodings of a pass's matrix.  The fused matrix arrives in FP64
// (complex128, row-major, sorted-target order) and is rounded exactly once
// to the pass precision here.
#include <cstring>

#include "sv_internal.h"

namespace sv {

size_t mfma_data_bytes(const Pass& p);
void mfma_encode(const Pass& p, const double* mat, unsigned char* dst);

size_t pass_data_bytes(const Pass& p) {
  if (p.variant == V_MFMA) return mfma_data_bytes(p);
  const size_t d = (size_t)1 << p.k;
  return d * d * 8;  // complex64
}

void encode_pass_data(const Pass& p, const double* mat, unsigned char* dst) {
  if (p.variant == V_MFMA) {
    mfma_encode(p, mat, dst);
    return;
  }
  const size_t d = (size_t)1 << p.k;
  float* f = reinterpret_cast<float*>(dst);
  for (size_t i = 0; i < 2 * d * d; ++i) f[i] = (float)mat[i];
}

}  // namespace sv
