#pragma once
// Launchers of the persistent sweep kernel, per precision (instantiated by
// stc_flow_f64.hip and stc_flow_f32.hip).
#include "stc_device.h"

namespace stc {

// persistent launch: one cooperative launch of G + 1 blocks per burst
template <typename T, int MP, int B, int RG, bool NT>
static int flow_resident_v() {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_flow<T, MP, B, RG, NT>,
                                                     kWG, 0) != hipSuccess)
        return 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

template <typename T, int MP, int B, int RG, bool NT>
static hipError_t flow_v(const FlowLaunch &f, hipStream_t s) {
    const int nflags = 2 * f.G + 2;
    hipError_t e = launch_flow_reset(f.flags, nflags, s);
    if (e != hipSuccess) return e;
    FlowLaunch arg = f;
    void *args[] = {(void *)&arg};
    return hipLaunchCooperativeKernel((const void *)k_sweep_flow<T, MP, B, RG, NT>,
                                      dim3(f.G + 1), dim3(kWG), args, 0, s);
}

template <typename T, int MP, int B>
static int flow_mpb(bool launch, int variant, const FlowLaunch *f, hipStream_t s,
                    hipError_t *err) {
    switch (variant & 3) {
        case 0:
            if (launch) *err = flow_v<T, MP, B, variant_rg(MP, 0), variant_nt(0)>(*f, s);
            return launch ? 0 : flow_resident_v<T, MP, B, variant_rg(MP, 0), variant_nt(0)>();
        case 1:
            if (launch) *err = flow_v<T, MP, B, variant_rg(MP, 1), variant_nt(1)>(*f, s);
            return launch ? 0 : flow_resident_v<T, MP, B, variant_rg(MP, 1), variant_nt(1)>();
        case 2:
            if (launch) *err = flow_v<T, MP, B, variant_rg(MP, 2), variant_nt(2)>(*f, s);
            return launch ? 0 : flow_resident_v<T, MP, B, variant_rg(MP, 2), variant_nt(2)>();
        default:
            if (launch) *err = flow_v<T, MP, B, variant_rg(MP, 3), variant_nt(3)>(*f, s);
            return launch ? 0 : flow_resident_v<T, MP, B, variant_rg(MP, 3), variant_nt(3)>();
    }
}

template <typename T, int B>
static int flow_b(int MP, bool launch, int variant, const FlowLaunch *f, hipStream_t s,
                  hipError_t *err) {
    switch (MP) {
        case 8: return flow_mpb<T, 8, B>(launch, variant, f, s, err);
        case 16: return flow_mpb<T, 16, B>(launch, variant, f, s, err);
        case 32: return flow_mpb<T, 32, B>(launch, variant, f, s, err);
        case 64: return flow_mpb<T, 64, B>(launch, variant, f, s, err);
        case 128: return flow_mpb<T, 128, B>(launch, variant, f, s, err);
    }
    *err = hipErrorInvalidValue;
    return 0;
}

// Block bandwidths 1 and 2 only: wider bands read levels of more than the
// neighbouring blocks, which the launch's waits are not laid out for.
template <typename T>
int flow_dispatch_t(int MP, int b, bool launch, int variant, const FlowLaunch *f, hipStream_t s,
                    hipError_t *err) {
    switch (b) {
        case 1: return flow_b<T, 1>(MP, launch, variant, f, s, err);
        case 2: return flow_b<T, 2>(MP, launch, variant, f, s, err);
    }
    *err = hipErrorInvalidValue;
    return 0;
}

}  // namespace stc
