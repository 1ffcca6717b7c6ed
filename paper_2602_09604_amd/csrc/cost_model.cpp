// Learned fusion cost model: features, host inference, partition search.
#include "sv_internal.h"

namespace sv {

void cost_features(int k, const int* qubits, int n, int precision, float* out) {
  for (int i = 0; i < SV_COST_FEATURES; ++i) out[i] = 0.f;
  out[0] = k / 6.0f;
  out[1] = n / 34.0f;
  for (int j = 0; j < k; ++j)
    if (qubits[j] < 34) out[2 + qubits[j]] = 1.f;
  if (precision >= 0 && precision < 4) out[36 + precision] = 1.f;
}
bool cost_model_ready() { return false; }
double cost_model_predict_log(int, const int*, int, int) { return 0.0; }
bool fuse_learned(const sv_gate*, size_t, int, int, int, std::vector<FusedGate>&, std::vector<int32_t>&) {
  return false;
}

}  // namespace sv

extern "C" {
int sv_cost_model_install(sv_mlp*) { return sv::fail(SV_EUNSUPPORTED, "cost model not built yet"); }
int sv_cost_model_save(const char*) { return sv::fail(SV_EUNSUPPORTED, "cost model not built yet"); }
int sv_cost_model_load(const char*) { return sv::fail(SV_EUNSUPPORTED, "cost model not built yet"); }
int sv_cost_model_predict(int, const int32_t*, int, int, double*) {
  return sv::fail(SV_EUNSUPPORTED, "cost model not built yet");
}
int sv_cost_features(int k, const int32_t* qubits, int n_qubits, int precision, float* out) {
  if (!qubits || !out || k < 1 || k > SV_MAX_K) return sv::fail(SV_EINVAL, "bad arguments");
  sv::cost_features(k, qubits, n_qubits, precision, out);
  return SV_OK;
}
}
