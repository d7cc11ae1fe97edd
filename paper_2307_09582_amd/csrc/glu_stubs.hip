// Entry points not yet implemented in this build report GLU_ERR_UNSUPPORTED.
#include "glu_host.h"

using namespace glu;

extern "C" {

glu_status glu_batch_plan_create(const glu_batch_item*, int32_t, const glu_params*, glu_batch_plan**) {
  return fail(GLU_ERR_UNSUPPORTED, "batch plans not built");
}
glu_status glu_batch_plan_launch(const glu_batch_plan*, void*) {
  return fail(GLU_ERR_UNSUPPORTED, "batch plans not built");
}
void glu_batch_plan_destroy(glu_batch_plan*) {}
glu_status glu_batch_plan_info(const glu_batch_plan*, int64_t*, int32_t*) {
  return fail(GLU_ERR_UNSUPPORTED, "batch plans not built");
}
glu_status glu_autotune(const glu_batch_item*, const glu_params*, int32_t*, void*) {
  return fail(GLU_ERR_UNSUPPORTED, "autotune not built");
}
glu_status glu_autotune_save(const char*) { return fail(GLU_ERR_UNSUPPORTED, "autotune not built"); }
glu_status glu_autotune_load(const char*) { return fail(GLU_ERR_UNSUPPORTED, "autotune not built"); }

}  // extern "C"
