// Sweep kernels of degree p = 4 (see sweep_device.h).
#include "sweep_device.h"

namespace vefk {

hipError_t launch_sweep_p4(const SweepLaunch &L, bool dir) {
  return dir ? launch_p<4, true>(L) : launch_p<4, false>(L);
}

hipError_t launch_class_inv_p4(const ClassInvLaunch &C) { return launch_class_p<4>(C); }

}  // namespace vefk
