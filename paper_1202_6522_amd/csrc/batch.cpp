// Batches of fields with different truncations: placeholder entry points,
// replaced by the batched implementation.
#include "shtn.h"

extern "C" {
shtn_batch_t shtn_batch(int, const shtn_plan_t*) { return nullptr; }
void shtn_batch_destroy(shtn_batch_t) {}
int shtn_batch_offsets(shtn_batch_t, size_t*, size_t*) { return SHTN_EUNSUPPORTED; }
size_t shtn_batch_device_bytes(shtn_batch_t) { return 0; }
size_t shtn_batch_work_bytes(shtn_batch_t) { return 0; }
int shtn_batch_upload(shtn_batch_t, void*, void*) { return SHTN_EUNSUPPORTED; }
int shtn_batch_synth(shtn_batch_t, const double*, double*, void*, void*) { return SHTN_EUNSUPPORTED; }
int shtn_batch_analys(shtn_batch_t, const double*, double*, void*, void*) { return SHTN_EUNSUPPORTED; }
int shtn_batch_set_tiling(shtn_batch_t, int, int, int, int) { return SHTN_EUNSUPPORTED; }
}
