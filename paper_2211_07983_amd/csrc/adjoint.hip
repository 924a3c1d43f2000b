// Reverse pass (filled in below).
#include "engine.h"
#include "plan_impl.h"

void plan_backward(mps_plan* p, double* grad, int on_device, mps_stats* stats) {
  (void)p; (void)grad; (void)on_device; (void)stats;
  fail(MPS_EINVAL, "reverse pass not built");
}
