// Launch-shape table: defaults, overridden by autotuner results.
#include "sv_internal.h"

namespace sv {

Shape tuned_shape(int variant, int n, int k, const int* s, int precision) {
  (void)variant; (void)n; (void)k; (void)s; (void)precision;
  Shape sh;
  sh.tile_bits = 12;
  sh.reg_iters = 1;
  sh.mfma_cols = 32;
  return sh;
}

}  // namespace sv

extern "C" {
int sv_autotune(sv_state*, int) { return sv::fail(SV_EUNSUPPORTED, "autotuner not built yet"); }
int sv_tune_save(const char*) { return sv::fail(SV_EUNSUPPORTED, "autotuner not built yet"); }
int sv_tune_load(const char*) { return sv::fail(SV_EUNSUPPORTED, "autotuner not built yet"); }
}
