// Entry points whose implementation lands in later files; each returns a
// clear error until then.
#include "stev_runtime.h"

void serve_stop(stev_ctx *) {}

extern "C" int stev_integrate_batched(stev_ctx *ctx, int32_t, const stev_mech *const *,
                                      const int64_t *, void *const *, const void *const *,
                                      void *const *, const int64_t *, const int64_t *, double,
                                      const stev_params *, int32_t *const *, uint8_t *const *,
                                      stev_stats *) {
  return stev_fail(ctx, STEV_EINVAL, "stev_integrate_batched: not built yet");
}
extern "C" int stev_submit(stev_ctx *ctx, const stev_mech *, int64_t, void *, const void *, void *,
                           int64_t, int64_t, double, const stev_params *, int32_t *, uint8_t *,
                           uint64_t *) {
  return stev_fail(ctx, STEV_EINVAL, "stev_submit: not built yet");
}
extern "C" int stev_poll(stev_ctx *ctx, uint64_t, stev_stats *) {
  return stev_fail(ctx, STEV_ENOTFOUND, "stev_poll: not built yet");
}
extern "C" int stev_autotune(stev_ctx *ctx, const stev_mech *, int64_t, const void *, const void *,
                             const void *, int64_t, int64_t, double, stev_params *) {
  return stev_fail(ctx, STEV_EINVAL, "stev_autotune: not built yet");
}
