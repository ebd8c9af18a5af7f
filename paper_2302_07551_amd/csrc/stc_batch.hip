// Dispatch of the multi-chain (batched) sweep launch to its per-precision
// launchers (stc_batch_f64.hip, stc_batch_f32.hip).
#include "stc_device.h"

namespace stc {

template <typename T>
hipError_t batch_phase_t(int b, int MP, bool phase_b, int variant, int grid,
                         const ChainDesc *chains, const WorkItem *items, const int *nitems,
                         int j, hipStream_t s);

hipError_t launch_batch_phase(int precision_bytes, int b, int MP, bool phase_b, int variant,
                              int grid, const ChainDesc *chains, const WorkItem *items,
                              const int *nitems, int j, hipStream_t stream) {
    if (variant < 0 || grid < 1 || j < 0) return hipErrorInvalidValue;
    return precision_bytes == 8
               ? batch_phase_t<double>(b, MP, phase_b, variant, grid, chains, items, nitems, j,
                                       stream)
               : batch_phase_t<float>(b, MP, phase_b, variant, grid, chains, items, nitems, j,
                                      stream);
}

}  // namespace stc
