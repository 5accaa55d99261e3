// batch.hip -- placeholder until the batched form is built.
#include "runtime.h"

extern "C" {
int imb_batch_required_bytes(int32_t, const imb_config*, size_t*) { return IMB_EUNSUPPORTED; }
int imb_batch_create(int32_t, const imb_config*, void*, void*, size_t, imb_batch** out) {
  if (out) *out = nullptr;
  return IMB_EUNSUPPORTED;
}
void imb_batch_destroy(imb_batch*) {}
int imb_batch_set_particles(imb_batch*, int32_t, int32_t, const double*, const double*,
                            const double*, const double*, const double*, const double*,
                            const int32_t*) { return IMB_EUNSUPPORTED; }
int imb_batch_step(imb_batch*, int32_t) { return IMB_EUNSUPPORTED; }
int imb_batch_get_forces(imb_batch*, int32_t, double*, double*, double*) { return IMB_EUNSUPPORTED; }
int imb_batch_get_particles(imb_batch*, int32_t, double*, double*, double*, double*, double*) {
  return IMB_EUNSUPPORTED;
}
int imb_batch_get_fields(imb_batch*, int32_t, double*, double*, double*) { return IMB_EUNSUPPORTED; }
int imb_batch_sync(imb_batch*) { return IMB_EUNSUPPORTED; }
int imb_batch_set_launch(imb_batch*, int32_t, int32_t, int32_t) { return IMB_EUNSUPPORTED; }
}
