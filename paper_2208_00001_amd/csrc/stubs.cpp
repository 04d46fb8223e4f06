// Entry points not yet implemented in this build: they validate nothing and
// report GGDT_ERR_UNSUPPORTED.
#include "ggdt.h"

extern "C" {

int ggdt2d_backward(const float*, const uint8_t*, const float*, const float*, float, float, int, float*, float*, int,
                    int, int, void*, size_t, hipStream_t) {
  return GGDT_ERR_UNSUPPORTED;
}
int ggdt3d_backward(const float*, const uint8_t*, const float*, const float*, float, float, int, float*, float*, int,
                    int, int, int, void*, size_t, hipStream_t) {
  return GGDT_ERR_UNSUPPORTED;
}
int ggdt_batched_plan(const ggdt_instance*, int, const ggdt_tuning*, ggdt_plan**, size_t*) {
  return GGDT_ERR_UNSUPPORTED;
}
int ggdt_batched_run(const ggdt_plan*, void*, size_t, hipStream_t) { return GGDT_ERR_UNSUPPORTED; }
int ggdt_batched_backward(const ggdt_plan*, void*, size_t, hipStream_t) { return GGDT_ERR_UNSUPPORTED; }
void ggdt_plan_destroy(ggdt_plan*) {}
}
