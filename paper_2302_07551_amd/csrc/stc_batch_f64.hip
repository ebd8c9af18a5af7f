// Batched sweep launchers, double blocks.
#include "stc_launch_batch.h"

namespace stc {
template hipError_t batch_phase_t<double>(int, int, bool, int, int, const ChainDesc *,
                                      const WorkItem *, const int *, int, hipStream_t);
}  // namespace stc
