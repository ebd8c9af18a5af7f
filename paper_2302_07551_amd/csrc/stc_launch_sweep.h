#pragma once
// Launchers of the dense sweep kernel, per precision (instantiated by
// stc_sweep_f64.hip and stc_sweep_f32.hip).
#include "stc_device.h"

namespace stc {

template <typename T, int MP, int B, int RG, bool NT>
static hipError_t sweep_v(bool phase_b, int variant, const SweepLaunch &a, hipStream_t s,
                          LaunchTimer t) {
    const int groups = phase_groups((int)sizeof(T), MP, a.L, a.parity, variant) +
                       ((phase_b && a.fold) ? 1 : 0);   // + the reduction workgroup
    if (groups <= 0) return hipSuccess;
    if (phase_b)
        launch_timed(k_sweep<T, MP, B, true, RG, NT>, groups, s, t, a);
    else
        launch_timed(k_sweep<T, MP, B, false, RG, NT>, groups, s, t, a);
    return hipGetLastError();
}

template <typename T, int MP, int B>
static hipError_t sweep_mpb(bool phase_b, int variant, const SweepLaunch &a, hipStream_t s,
                            LaunchTimer t) {
    switch (variant & 3) {   // bit 2 (persistent bursts) has the same phases
        case 0: return sweep_v<T, MP, B, variant_rg(MP, 0), variant_nt(0)>(phase_b, 0, a, s, t);
        case 1: return sweep_v<T, MP, B, variant_rg(MP, 1), variant_nt(1)>(phase_b, 1, a, s, t);
        case 2: return sweep_v<T, MP, B, variant_rg(MP, 2), variant_nt(2)>(phase_b, 2, a, s, t);
        case 3: return sweep_v<T, MP, B, variant_rg(MP, 3), variant_nt(3)>(phase_b, 3, a, s, t);
    }
    return hipErrorInvalidValue;
}

template <typename T, int B>
static hipError_t sweep_b(int MP, bool phase_b, int variant, const SweepLaunch &a,
                          hipStream_t s, LaunchTimer t) {
    switch (MP) {
        case 8: return sweep_mpb<T, 8, B>(phase_b, variant, a, s, t);
        case 16: return sweep_mpb<T, 16, B>(phase_b, variant, a, s, t);
        case 32: return sweep_mpb<T, 32, B>(phase_b, variant, a, s, t);
        case 64: return sweep_mpb<T, 64, B>(phase_b, variant, a, s, t);
        case 128: return sweep_mpb<T, 128, B>(phase_b, variant, a, s, t);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t sweep_phase_t(int MP, int b, bool phase_b, int variant, const SweepLaunch &a,
                         hipStream_t s, LaunchTimer t) {
    switch (b) {
        case 1: return sweep_b<T, 1>(MP, phase_b, variant, a, s, t);
        case 2: return sweep_b<T, 2>(MP, phase_b, variant, a, s, t);
        case 3: return sweep_b<T, 3>(MP, phase_b, variant, a, s, t);
        case 4: return sweep_b<T, 4>(MP, phase_b, variant, a, s, t);
    }
    return hipErrorInvalidValue;
}

}  // namespace stc
