#pragma once
// Launchers of the multi-chain (batched) sweep kernel, per precision
// (instantiated by stc_batch_f64.hip and stc_batch_f32.hip).
#include "stc_device.h"

namespace stc {

template <typename T, int MP, int B, int RG, bool NT>
static hipError_t batch_v(bool phase_b, int grid, const ChainDesc *chains, const WorkItem *items,
                          const int *nitems, int j, hipStream_t s) {
    if (phase_b)
        hipLaunchKernelGGL((k_batch_sweep<T, MP, B, true, RG, NT>), dim3(grid), dim3(kWG), 0, s,
                           chains, items, nitems, j);
    else
        hipLaunchKernelGGL((k_batch_sweep<T, MP, B, false, RG, NT>), dim3(grid), dim3(kWG), 0, s,
                           chains, items, nitems, j);
    return hipGetLastError();
}

template <typename T, int MP, int B>
static hipError_t batch_mpb(bool phase_b, int variant, int grid, const ChainDesc *chains,
                            const WorkItem *items, const int *nitems, int j, hipStream_t s) {
    switch (variant & 3) {
        case 0:
            return batch_v<T, MP, B, variant_rg(MP, 0), variant_nt(0)>(phase_b, grid, chains,
                                                                       items, nitems, j, s);
        case 1:
            return batch_v<T, MP, B, variant_rg(MP, 1), variant_nt(1)>(phase_b, grid, chains,
                                                                       items, nitems, j, s);
        case 2:
            return batch_v<T, MP, B, variant_rg(MP, 2), variant_nt(2)>(phase_b, grid, chains,
                                                                       items, nitems, j, s);
        default:
            return batch_v<T, MP, B, variant_rg(MP, 3), variant_nt(3)>(phase_b, grid, chains,
                                                                       items, nitems, j, s);
    }
}

template <typename T, int B>
static hipError_t batch_b(int MP, bool phase_b, int variant, int grid, const ChainDesc *chains,
                          const WorkItem *items, const int *nitems, int j, hipStream_t s) {
    switch (MP) {
        case 8: return batch_mpb<T, 8, B>(phase_b, variant, grid, chains, items, nitems, j, s);
        case 16: return batch_mpb<T, 16, B>(phase_b, variant, grid, chains, items, nitems, j, s);
        case 32: return batch_mpb<T, 32, B>(phase_b, variant, grid, chains, items, nitems, j, s);
        case 64: return batch_mpb<T, 64, B>(phase_b, variant, grid, chains, items, nitems, j, s);
        case 128: return batch_mpb<T, 128, B>(phase_b, variant, grid, chains, items, nitems, j, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t batch_phase_t(int b, int MP, bool phase_b, int variant, int grid,
                         const ChainDesc *chains, const WorkItem *items, const int *nitems,
                         int j, hipStream_t s) {
    switch (b) {
        case 1: return batch_b<T, 1>(MP, phase_b, variant, grid, chains, items, nitems, j, s);
        case 2: return batch_b<T, 2>(MP, phase_b, variant, grid, chains, items, nitems, j, s);
        case 3: return batch_b<T, 3>(MP, phase_b, variant, grid, chains, items, nitems, j, s);
        case 4: return batch_b<T, 4>(MP, phase_b, variant, grid, chains, items, nitems, j, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace stc
