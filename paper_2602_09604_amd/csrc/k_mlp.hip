// MLP cost-model kernels (forward, backward, Adam).
#include "sv_internal.h"

extern "C" {
int sv_mlp_create(int, uint64_t, void*, sv_mlp** out) { if (out) *out = nullptr; return sv::fail(SV_EUNSUPPORTED, "mlp not built yet"); }
int sv_mlp_free(sv_mlp*) { return SV_OK; }
int sv_mlp_num_params(const sv_mlp*, size_t*) { return sv::fail(SV_EUNSUPPORTED, "mlp not built yet"); }
int sv_mlp_get_params(sv_mlp*, float*) { return sv::fail(SV_EUNSUPPORTED, "mlp not built yet"); }
int sv_mlp_set_params(sv_mlp*, const float*) { return sv::fail(SV_EUNSUPPORTED, "mlp not built yet"); }
int sv_mlp_forward(sv_mlp*, const float*, int, float*) { return sv::fail(SV_EUNSUPPORTED, "mlp not built yet"); }
int sv_mlp_loss_grad(sv_mlp*, const float*, const float*, int, float*, float*) { return sv::fail(SV_EUNSUPPORTED, "mlp not built yet"); }
int sv_mlp_adam_step(sv_mlp*, float, float, float, float) { return sv::fail(SV_EUNSUPPORTED, "mlp not built yet"); }
int sv_mlp_train(sv_mlp*, const float*, const float*, int, int, float, float*) { return sv::fail(SV_EUNSUPPORTED, "mlp not built yet"); }
}
