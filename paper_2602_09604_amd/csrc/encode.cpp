// Device encodings of a pass's matrix.  The fused matrix arrives in FP64
// (complex128, row-major, sorted-target order) and is rounded exactly once
// to the pass precision here.
#include <cstring>

#include "sv_internal.h"

namespace sv {

size_t mfma_data_bytes(const Pass& p);
void mfma_encode(const Pass& p, const double* mat, unsigned char* dst);

// Register passes (no controls) also carry the matrix in the 3M form the
// register kernel multiplies with up to four element-space targets: per
// element ur, ur + ui, ui - ur (formed in FP64, then rounded), after the
// complex64 copy the other forms read.
static bool has_3m(const Pass& p) { return p.variant == V_REG && p.cmask == 0; }

size_t pass_data_bytes(const Pass& p) {
  if (p.variant == V_MFMA) return mfma_data_bytes(p);
  const size_t d = (size_t)1 << p.k;
  return d * d * (has_3m(p) ? 20 : 8);  // complex64 (+ three floats per element)
}

void encode_pass_data(const Pass& p, const double* mat, unsigned char* dst) {
  if (p.variant == V_MFMA) {
    mfma_encode(p, mat, dst);
    return;
  }
  const size_t d = (size_t)1 << p.k;
  float* f = reinterpret_cast<float*>(dst);
  for (size_t i = 0; i < 2 * d * d; ++i) f[i] = (float)mat[i];
  if (!has_3m(p)) return;
  float* g = f + 2 * d * d;
  for (size_t e = 0; e < d * d; ++e) {
    const double ur = mat[2 * e], ui = mat[2 * e + 1];
    g[3 * e] = (float)ur;
    g[3 * e + 1] = (float)(ur + ui);
    g[3 * e + 2] = (float)(ui - ur);
  }
}

}  // namespace sv
