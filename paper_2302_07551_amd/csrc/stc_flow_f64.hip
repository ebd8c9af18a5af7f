// Persistent sweep launchers, double blocks.
#include "stc_launch_flow.h"

namespace stc {
template int flow_dispatch_t<double>(int, int, bool, int, const FlowLaunch *, hipStream_t,
                                  hipError_t *);
}  // namespace stc
