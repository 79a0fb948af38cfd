// Batched ensembles: placeholder until the persistent kernel lands.
#include "grf_internal.h"

struct grf_plan {
    int method;
};

extern "C" {
int grf_plan_create(grf_plan** plan, int, int, const char*)
{
    if (!plan) return grf::fail(GRF_EINVAL, "grf_plan_create: plan is NULL");
    *plan = nullptr;
    return grf::fail(GRF_EUNSUPPORTED, "grf_plan_create: not available yet");
}
int grf_plan_destroy(grf_plan*) { return GRF_OK; }
int eval_field_batch(grf_plan*, const grf_batch_item*, int32_t, void*)
{
    return grf::fail(GRF_EUNSUPPORTED, "eval_field_batch: not available yet");
}
int grf_plan_info(const grf_plan*, int32_t*, int32_t*, int32_t*, int64_t*)
{
    return grf::fail(GRF_EUNSUPPORTED, "grf_plan_info: not available yet");
}
}
