// Rank predictor (filled in below).
#include "runtime.h"

namespace smps { void mlp_free(smps_ctx*) {} }

extern "C" {
int smps_rank_mlp_init(smps_ctx*, unsigned long long) { return SMPS_EUNSUPPORTED; }
int smps_rank_mlp_train(smps_ctx*, int, const float*, const float*, int, int, float, float*) { return SMPS_EUNSUPPORTED; }
int smps_rank_mlp_predict(smps_ctx*, int, const float*, float*) { return SMPS_EUNSUPPORTED; }
int smps_rank_mlp_get(const smps_ctx*, float*, int) { return SMPS_EUNSUPPORTED; }
int smps_rank_mlp_set(smps_ctx*, const float*, int) { return SMPS_EUNSUPPORTED; }
int smps_rank_mlp_grad(smps_ctx*, int, const float*, const float*, float*, float*, int) { return SMPS_EUNSUPPORTED; }
}
