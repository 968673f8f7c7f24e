// Entry points whose kernels are not built yet: they validate nothing and
// report BZ_ERR_UNSUPPORTED.
#include "common.h"

using namespace bzi;

extern "C" {
int bz_eval_tensor_patch(const void *, int, int64_t, int, int, int, int, const float *, int64_t, int, int, int,
                         float *, bz_stream) { return fail(BZ_ERR_UNSUPPORTED, "bz_eval_tensor_patch: not built"); }
int bz_batch_plan_create(int64_t, const uint16_t *, const int64_t *, const void *, const void *, int, int,
                         const int64_t *, const float *, int64_t, int, bz_stream, bz_plan *) {
    return fail(BZ_ERR_UNSUPPORTED, "bz_batch_plan_create: not built");
}
int bz_batch_eval(bz_plan, const float *, float *, bz_stream) { return fail(BZ_ERR_UNSUPPORTED, "not built"); }
int bz_batch_plan_info(bz_plan, int64_t *) { return fail(BZ_ERR_UNSUPPORTED, "not built"); }
int bz_plan_destroy(bz_plan) { return BZ_OK; }
int bz_adjoint_bezier(const float *, const float *, int64_t, int, int, const float *, int64_t, int, const float *,
                      float *, float *, float *, bz_stream) { return fail(BZ_ERR_UNSUPPORTED, "not built"); }
int bz_fit_adam_step(float *, float *, const float *, int64_t, int, int, int64_t, float *, float *, float *, float *,
                     int, float, float, float, float, float *, bz_stream) { return fail(BZ_ERR_UNSUPPORTED, "not built"); }
int bz_fit_adam_run(float *, float *, const float *, int64_t, int, int, int64_t, float *, float *, float *, float *,
                    int, int, float, float, float, float, float *, bz_stream) { return fail(BZ_ERR_UNSUPPORTED, "not built"); }
}
