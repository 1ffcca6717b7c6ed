// Matrix-core passes for fused gates with k >= 4.
#include "sv_internal.h"

namespace sv {

bool mfma_supported(int k, int precision) { (void)k; (void)precision; return false; }
size_t mfma_data_bytes(const Pass& p) { const size_t d = (size_t)1 << p.k; return d * d * 8; }
void mfma_encode(const Pass& p, const double* mat, unsigned char* dst) {
  const size_t d = (size_t)1 << p.k;
  float* f = reinterpret_cast<float*>(dst);
  for (size_t i = 0; i < 2 * d * d; ++i) f[i] = (float)mat[i];
}
void launch_mfma(const Pass&, int, void*, const unsigned char*, hipStream_t) {
  throw DeviceError{hipErrorInvalidValue, "MFMA pass not built yet"};
}

}  // namespace sv
