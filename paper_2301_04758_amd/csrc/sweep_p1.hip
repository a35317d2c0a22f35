// Sweep kernels of degree p = 1 (see sweep_device.h).
#include "sweep_device.h"

namespace vefk {

hipError_t launch_sweep_p1(const SweepLaunch &L, bool dir) {
  return dir ? launch_p<1, true>(L) : launch_p<1, false>(L);
}

}  // namespace vefk
