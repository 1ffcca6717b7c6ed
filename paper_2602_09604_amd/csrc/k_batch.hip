// Batched persistent kernel for many small circuits.
#include "sv_internal.h"

extern "C" int sv_batch_run(sv_state* const*, const sv_gate* const*, const size_t*, size_t, const sv_run_opts*,
                            sv_run_stats*) {
  return sv::fail(SV_EUNSUPPORTED, "batched kernel not built yet");
}
