// Batched plans (persistent work-list launches).
#include "haar.h"
#include "haar_internal.h"

using namespace haar;

extern "C" {
int haar_plan_create_1d(const haar_item_1d*, int64_t, int32_t, int32_t, haar_plan** out) {
    if (out) *out = nullptr;
    return set_error(HAAR_ERR_UNSUPPORTED, "plans not built yet");
}
int haar_plan_create_2d(const haar_item_2d*, int64_t, int32_t, int32_t, haar_plan** out) {
    if (out) *out = nullptr;
    return set_error(HAAR_ERR_UNSUPPORTED, "plans not built yet");
}
int haar_plan_workspace_size(const haar_plan*, size_t*) { return set_error(HAAR_ERR_PLAN, "no plan"); }
int haar_plan_upload(haar_plan*, void*, void*) { return set_error(HAAR_ERR_PLAN, "no plan"); }
int haar_plan_execute(const haar_plan*, void*, void*) { return set_error(HAAR_ERR_PLAN, "no plan"); }
int haar_plan_info(const haar_plan*, int64_t*, int32_t*) { return set_error(HAAR_ERR_PLAN, "no plan"); }
int haar_plan_destroy(haar_plan*) { return HAAR_OK; }
}
