// Sweep kernels of degree p = 2 (see sweep_device.h).
#include "sweep_device.h"

namespace vefk {

hipError_t launch_sweep_p2(const SweepLaunch &L, bool dir) {
  return dir ? launch_p<2, true>(L) : launch_p<2, false>(L);
}

}  // namespace vefk
