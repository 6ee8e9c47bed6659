// Panther++ (placeholder until the feature and distance kernels land).
#include "../../include/panther.h"
#include "runtime.h"

void free_pp_state(panther_ctx* c) { (void)c; }

extern "C" int panther_pp_topk(panther_ctx* c, const int32_t*, int64_t, int32_t, int32_t,
                               int32_t*, double*, int, void*) {
  return ctx_fail(c, PANTHER_EINVAL, "Panther++ not built yet");
}
extern "C" int panther_get_features(panther_ctx* c, int32_t, float*, int) {
  return ctx_fail(c, PANTHER_EINVAL, "Panther++ not built yet");
}
extern "C" int panther_pp_stats(panther_ctx* c, double*, double*) {
  return ctx_fail(c, PANTHER_ESTATE, "no BF16 Panther++ call yet");
}
