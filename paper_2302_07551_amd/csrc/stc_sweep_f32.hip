// Dense sweep launchers, float blocks.
#include "stc_launch_sweep.h"

namespace stc {
template hipError_t sweep_phase_t<float>(int, int, bool, int, const SweepLaunch &, hipStream_t,
                                       LaunchTimer);
}  // namespace stc
