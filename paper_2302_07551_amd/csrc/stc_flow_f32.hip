// Persistent sweep launchers, float blocks.
#include "stc_launch_flow.h"

namespace stc {
template int flow_dispatch_t<float>(int, int, bool, int, const FlowLaunch *, hipStream_t,
                                  hipError_t *);
}  // namespace stc
