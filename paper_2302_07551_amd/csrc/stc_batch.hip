// Launchers of the multi-chain (batched) sweep kernel.
#include "stc_device.h"

namespace stc {

int batch_lpw(int precision_bytes, int MP) {
    return precision_bytes == 8 ? lpw_of<double>(MP, 0) : lpw_of<float>(MP, 0);
}

template <typename T, int MP, int B>
static hipError_t batch_mp(bool phase_b, bool nt, int grid, const ChainDesc *chains,
                           const WorkItem *items, const int *nitems, hipStream_t s) {
    if (phase_b) {
        if (nt)
            hipLaunchKernelGGL((k_batch_sweep<T, MP, B, true, true>), dim3(grid), dim3(kWG), 0, s,
                               chains, items, nitems);
        else
            hipLaunchKernelGGL((k_batch_sweep<T, MP, B, true, false>), dim3(grid), dim3(kWG), 0,
                               s, chains, items, nitems);
    } else {
        if (nt)
            hipLaunchKernelGGL((k_batch_sweep<T, MP, B, false, true>), dim3(grid), dim3(kWG), 0,
                               s, chains, items, nitems);
        else
            hipLaunchKernelGGL((k_batch_sweep<T, MP, B, false, false>), dim3(grid), dim3(kWG), 0,
                               s, chains, items, nitems);
    }
    return hipGetLastError();
}

template <typename T, int B>
static hipError_t batch_tb(int MP, bool phase_b, bool nt, int grid, const ChainDesc *chains,
                           const WorkItem *items, const int *nitems, hipStream_t s) {
    switch (MP) {
        case 8: return batch_mp<T, 8, B>(phase_b, nt, grid, chains, items, nitems, s);
        case 16: return batch_mp<T, 16, B>(phase_b, nt, grid, chains, items, nitems, s);
        case 32: return batch_mp<T, 32, B>(phase_b, nt, grid, chains, items, nitems, s);
        case 64: return batch_mp<T, 64, B>(phase_b, nt, grid, chains, items, nitems, s);
        case 128: return batch_mp<T, 128, B>(phase_b, nt, grid, chains, items, nitems, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batch_phase(int precision_bytes, int b, int MP, bool phase_b, bool nt, int grid,
                              const ChainDesc *chains, const WorkItem *items, const int *nitems,
                              hipStream_t stream) {
    const bool f64 = precision_bytes == 8;
    switch (b) {
        case 1: return f64 ? batch_tb<double, 1>(MP, phase_b, nt, grid, chains, items, nitems, stream)
                           : batch_tb<float, 1>(MP, phase_b, nt, grid, chains, items, nitems, stream);
        case 2: return f64 ? batch_tb<double, 2>(MP, phase_b, nt, grid, chains, items, nitems, stream)
                           : batch_tb<float, 2>(MP, phase_b, nt, grid, chains, items, nitems, stream);
        case 3: return f64 ? batch_tb<double, 3>(MP, phase_b, nt, grid, chains, items, nitems, stream)
                           : batch_tb<float, 3>(MP, phase_b, nt, grid, chains, items, nitems, stream);
        case 4: return f64 ? batch_tb<double, 4>(MP, phase_b, nt, grid, chains, items, nitems, stream)
                           : batch_tb<float, 4>(MP, phase_b, nt, grid, chains, items, nitems, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace stc
