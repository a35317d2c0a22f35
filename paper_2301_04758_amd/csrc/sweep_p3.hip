// Sweep kernels of degree p = 3 (see sweep_device.h).
#include "sweep_device.h"

namespace vefk {

hipError_t launch_sweep_p3(const SweepLaunch &L, bool dir) {
  return dir ? launch_p<3, true>(L) : launch_p<3, false>(L);
}

hipError_t launch_class_inv_p3(const ClassInvLaunch &C) { return launch_class_p<3>(C); }

hipError_t launch_pivot_order_p3(const PivotOrderLaunch &L) {
  return L.fp32 ? launch_pivot_order_t<3, float>(L) : launch_pivot_order_t<3, double>(L);
}

}  // namespace vefk
