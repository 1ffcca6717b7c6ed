// Host planning of passes: target normalisation, variant choice, LDS tile
// split, and the encoding of a pass's matrix for the device.
#include <algorithm>
#include <cstring>

#include "sv_internal.h"

namespace sv {

// Sort the targets ascending and permute the matrix to match: new local bit j
// is state bit sorted[j]; old local index = sum_j bit_j(new) << perm[j].
void normalise_gate(int k, const int32_t* qubits, const double* mat, int* sorted_out,
                    std::vector<double>& mat_out) {
  int perm[SV_MAX_K];
  for (int j = 0; j < k; ++j) perm[j] = j;
  std::sort(perm, perm + k, [&](int a, int b) { return qubits[a] < qubits[b]; });
  for (int j = 0; j < k; ++j) sorted_out[j] = qubits[perm[j]];
  const int d = 1 << k;
  std::vector<int> old_of(d);
  for (int l = 0; l < d; ++l) {
    int o = 0;
    for (int j = 0; j < k; ++j)
      if ((l >> j) & 1) o |= 1 << perm[j];
    old_of[l] = o;
  }
  mat_out.assign((size_t)2 * d * d, 0.0);
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      const size_t src = (size_t)2 * (old_of[r] * d + old_of[c]);
      const size_t dst = (size_t)2 * (r * d + c);
      mat_out[dst] = mat[src];
      mat_out[dst + 1] = mat[src + 1];
    }
}

// Number h of targets that fall at or above the chunk boundary m = T - h
// (the fixed point exists because #targets >= m is non-increasing in m).
int lds_split(int tile_bits, int k, const int* s, int* m_out) {
  for (int h = 0; h <= k; ++h) {
    const int m = tile_bits - h;
    int c = 0;
    for (int j = 0; j < k; ++j)
      if (s[j] >= m) ++c;
    if (c == h) {
      *m_out = m;
      return h;
    }
  }
  *m_out = tile_bits - k;
  return k;
}

// A target in bits 1..6 breaks the 1 KiB contiguous wavefront row of the
// register kernel (bit 0 is handled inside its 16-byte element).
static bool has_low_target(int k, const int* s) {
  for (int j = 0; j < k; ++j)
    if (s[j] >= 1 && s[j] < 7) return true;
  return false;
}

// The LDS kernel is built for tiles of 2^8, 2^10 and 2^12 amplitudes; with
// k <= 6 the chunk bits m = T - h stay >= 2, so any state of >= 8 qubits fits.
static bool lds_feasible(int n, int k, const int* s, int tile_bits) {
  (void)s;
  (void)tile_bits;
  return n >= 8 && k <= SV_MAX_K;
}

int tuned_variant(int n, int k, const int* s, int precision);

int choose_variant(int n, int k, const int* s, int precision, int requested) {
  const Shape sh = tuned_shape(V_LDS, n, k, s, precision);
  const bool mfma_ok = mfma_supported(k, precision) && n >= k + 6;
  if (requested == V_MFMA) return mfma_ok ? V_MFMA : V_REG;
  if (requested == V_LDS) return lds_feasible(n, k, s, sh.tile_bits) ? V_LDS : V_REG;
  if (requested == V_REG) return V_REG;
  const bool shfl_ok = shfl_eligible(n, k, s);
  if (requested == V_SHFL) return shfl_ok ? V_SHFL : V_REG;
  // AUTO: the autotuner's measurement for this pass class when there is one
  const int tv = tuned_variant(n, k, s, precision);
  if (tv == V_SHFL && shfl_ok) return V_SHFL;
  if (tv == V_MFMA && mfma_ok) return V_MFMA;
  if (tv == V_LDS && lds_feasible(n, k, s, sh.tile_bits)) return V_LDS;
  if (tv == V_REG) return V_REG;
  // untuned defaults, from sweeps at 30 and 32 qubits: matrix cores for k >= 4
  // when the precision asks for them; the wavefront shuffle for k <= 2 with
  // every target in bits 0..6; on streamed states the register kernel
  // whenever it reads whole lines (its lane exchange covers targets on bits
  // 1..3): 0.68-0.76 of peak against 0.49-0.65 for LDS staging on every
  // low-target set measured; LDS staging for other low targets up to k = 4
  if (precision != SV_PREC_FP32_VALU && mfma_ok) return V_MFMA;
  if (shfl_ok && k <= 2) return V_SHFL;  // at k = 3 the permutes cost more; only when tuned
  if (reg_streams(n, k, s)) return V_REG;
  if (has_low_target(k, s) && k <= 4 && lds_feasible(n, k, s, sh.tile_bits)) return V_LDS;
  return V_REG;
}

}  // namespace sv
