// Kernels without template parameters and the launchers that are not split
// per precision: the state, reduction, load and store, residual, change,
// inverse and sparse-sweep launches, and the dispatch to the per-precision
// launcher files.
#include "stc_device.h"

namespace stc {

__global__ void k_flow_reset(unsigned *flags, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        flags[i] = 0u;
}



__global__ __launch_bounds__(kWG) void k_finalize_sweep(const double *part_sum,
                                                         const double *part_diff, int nslots,
                                                         DevState *st, long long s, double tol) {
    __shared__ double sh[4 * kWG / 64];
    finalize_chain(part_sum, part_diff, nslots, st, s, tol, sh);
}

// The finalize of sweep burst_base + j of a batch's chains chains[range[0]
// .. range[0] + range[1] - 1], one workgroup per chain (the range is read on
// the device, so a captured graph stays valid when the membership changes).
__global__ __launch_bounds__(kWG) void k_batch_finalize(const ChainDesc *chains,
                                                         const int *range, int j) {
    __shared__ double sh[4 * kWG / 64];
    if ((int)blockIdx.x >= range[1]) return;
    const ChainDesc &d = chains[range[0] + blockIdx.x];
    DevState *st = d.st;
    const long long s = st->burst_base + j;
    const size_t p = (size_t)(s & 1) * d.nparts;
    finalize_chain(d.part_sum + p, d.part_diff + p, d.groups_a + d.groups_b, st, s, d.tol, sh);
}

// Start of a burst of batched sweeps: each chain's sweeps are numbered from
// the one after its last recorded sweep (one thread per chain).
__global__ __launch_bounds__(kWG) void k_batch_begin(const ChainDesc *chains, const int *range) {
    const int c = blockIdx.x * kWG + threadIdx.x;
    if (c >= range[1]) return;
    DevState *st = chains[range[0] + c].st;
    st->burst_base = st->last_sweep + 1;
}



// Gather the stopping state of n chains into one table (one thread per
// chain).  The change reported is that of the stop sweep once stopped, else
// of the sweep two back: lagged normalisation measures it two sweeps late.
__global__ __launch_bounds__(kWG) void k_batch_query(DevState *const *states, int n,
                                                      QueryRow *out) {
    const int c = blockIdx.x * kWG + threadIdx.x;
    if (c >= n) return;
    const DevState *st = states[c];
    const int f = st->stop_flag;
    const long long ls = st->last_sweep;
    const long long k = f ? st->stop_sweep : ls - 2;
    QueryRow r;
    r.sweeps = f ? st->stop_sweep : ls;
    r.last_sweep = ls;
    r.diff = k >= 1 ? st->diff[k & kRingMask] : INFINITY;
    r.stopped = f;
    r.status = st->status;
    out[c] = r;
}



// Continue from sweep k after a precision switch: clear the stop state.
__global__ void k_rearm(DevState *st, long long k) {
    if (threadIdx.x == 0) {
        st->stop_flag = 0;
        st->status = kDevOk;
        st->stop_sweep = -1;
        st->last_sweep = k;
        st->test_after = k;
    }
}



// mode kReduceResidual writes the sum to *out, or to DevState::residual when
// out is null.
__global__ __launch_bounds__(kWG) void k_reduce(const double *part, int n, int mode,
                                                 DevState *st, long long slot, double tol,
                                                 double *out) {
    __shared__ double sh[4 * kWG / 64];
    const int stride = (mode == kReduceLoad) ? 2 : 1;
    double t = 0.0, tc = 0.0, b = 0.0;
    for (int j = threadIdx.x; j < n; j += kWG) {
        dd_acc(t, tc, part[stride * j]);
        if (mode == kReduceLoad) b = fmax(b, part[2 * j + 1]);
    }
    t = block_sum_dd(t, tc, sh);
    if (mode == kReduceLoad) b = block_max(b, sh);
    if (threadIdx.x != 0) return;
    if (mode == kReduceResidual) {
        if (out)
            *out = t;
        else
            st->residual = t;
    } else if (mode == kReduceDiff) {
        // the change of sweep slot, with the device stopping test
        if (st->stop_flag || slot <= st->test_after) return;
        st->diff[slot & kRingMask] = t;
        if (tol > 0.0 && t <= tol) {
            st->stop_flag = 1;
            st->stop_sweep = slot;
        }
    } else {
        st->x_sum = t;
        // slot < 0: a raw vector for the residual, no start-vector checks
        if (slot >= 0) {
            if (b > 0.0 || !(t > 0.0) || !isfinite(t)) {
                st->status = kDevBadStart;
                st->inv_sigma[slot & kRingMask] = 0.0;
            } else {
                st->inv_sigma[slot & kRingMask] = 1.0 / t;
                // the first sweep's input scale kappa_1 = 1 / e^T W_0 as well
                if (slot == 0) st->inv_sigma[kRingMask] = 1.0 / t;
            }
        }
    }
}



__global__ __launch_bounds__(kWG) void k_cast(const double *src, float *dst, size_t n) {
    for (size_t j = blockIdx.x * (size_t)kWG + threadIdx.x; j < n; j += (size_t)gridDim.x * kWG)
        dst[j] = (float)src[j];
}



__global__ __launch_bounds__(kWG) void k_widen(const float *src, double *dst, size_t n) {
    for (size_t j = blockIdx.x * (size_t)kWG + threadIdx.x; j < n; j += (size_t)gridDim.x * kWG)
        dst[j] = (double)src[j];
}



__global__ void k_reset(DevState *st) {
    if (threadIdx.x == 0) {
        st->stop_flag = 0;
        st->status = kDevOk;
        st->stop_sweep = -1;
        st->last_sweep = 0;
        st->residual = 0.0;
        st->test_after = 0;
        st->burst_base = 1;
    }
}



// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int supported_mp(int m) {
    if (m < 1 || m > kMaxMP) return 0;
    int mp = 8;
    while (mp < m) mp <<= 1;
    return mp;
}


int variant_count() { return kVariants; }

int phase_groups(int precision_bytes, int MP, int L, int parity, int variant) {
    const int levels = (L - parity + 1) / 2;
    if (MP > kMaxSmallMP) return levels * big_slices(precision_bytes, MP);
    const int lpw = precision_bytes == 8 ? lpw_of<double>(MP, variant) : lpw_of<float>(MP, variant);
    return (levels + lpw - 1) / lpw;
}

int reduce_groups(int MP, int L) {
    if (MP > kMaxSmallMP) return L * big_residual_slices(MP);
    const int lpw = lpw_of<double>(MP, kEllGeometry);   // the residual kernel's 8-row-group tile
    return (L + lpw - 1) / lpw;
}


hipError_t launch_sweep_phase(int precision_bytes, int MP, int b, bool phase_b, int variant,
                              const SweepLaunch &a, hipStream_t stream, LaunchTimer t) {
    if (variant < 0 || variant >= kVariants) return hipErrorInvalidValue;
    return precision_bytes == 8 ? sweep_phase_t<double>(MP, b, phase_b, variant, a, stream, t)
                                : sweep_phase_t<float>(MP, b, phase_b, variant, a, stream, t);
}

hipError_t launch_flow_reset(unsigned *flags, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_flow_reset, dim3((n + kWG - 1) / kWG), dim3(kWG), 0, s, flags, n);
    return hipGetLastError();
}

static int flow_dispatch(int precision_bytes, int MP, int b, bool launch, int variant,
                         const FlowLaunch *f, hipStream_t s, hipError_t *err) {
    return precision_bytes == 8 ? flow_dispatch_t<double>(MP, b, launch, variant, f, s, err)
                                : flow_dispatch_t<float>(MP, b, launch, variant, f, s, err);
}

int flow_resident_blocks(int precision_bytes, int MP, int b, int variant) {
    hipError_t e = hipSuccess;
    return flow_dispatch(precision_bytes, MP, b, false, variant, nullptr, nullptr, &e);
}

hipError_t launch_sweep_flow(int precision_bytes, int MP, int b, int variant, const FlowLaunch &f,
                             hipStream_t stream) {
    if (f.G < 1 || f.n < 1) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    flow_dispatch(precision_bytes, MP, b, true, variant, &f, stream, &e);
    return e;
}

template <typename T, int MP, int B>
static hipError_t ell_mpb(bool phase_b, const SweepLaunch &a, const EllEntry *tab,
                          const void *val, const unsigned char *idx, hipStream_t s,
                          LaunchTimer t) {
    const int groups = phase_groups((int)sizeof(T), MP, a.L, a.parity, kEllGeometry) +
                       ((phase_b && a.fold) ? 1 : 0);
    if (groups <= 0) return hipSuccess;
    if (phase_b)
        launch_timed(k_sweep_ell<T, MP, B, true>, groups, s, t, a, tab, val, idx);
    else
        launch_timed(k_sweep_ell<T, MP, B, false>, groups, s, t, a, tab, val, idx);
    return hipGetLastError();
}

template <typename T, int B>
static hipError_t ell_b(int MP, bool phase_b, const SweepLaunch &a, const EllEntry *tab,
                        const void *val, const unsigned char *idx, hipStream_t s,
                        LaunchTimer t) {
    switch (MP) {
        case 8: return ell_mpb<T, 8, B>(phase_b, a, tab, val, idx, s, t);
        case 16: return ell_mpb<T, 16, B>(phase_b, a, tab, val, idx, s, t);
        case 32: return ell_mpb<T, 32, B>(phase_b, a, tab, val, idx, s, t);
        case 64: return ell_mpb<T, 64, B>(phase_b, a, tab, val, idx, s, t);
        case 128: return ell_mpb<T, 128, B>(phase_b, a, tab, val, idx, s, t);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_phase_ell(int precision_bytes, int MP, int b, bool phase_b,
                                  const SweepLaunch &a, const EllEntry *tab, const void *val,
                                  const unsigned char *idx, hipStream_t stream, LaunchTimer t) {
    const bool f64 = precision_bytes == 8;
    switch (b) {
        case 1: return f64 ? ell_b<double, 1>(MP, phase_b, a, tab, val, idx, stream, t)
                           : ell_b<float, 1>(MP, phase_b, a, tab, val, idx, stream, t);
        case 2: return f64 ? ell_b<double, 2>(MP, phase_b, a, tab, val, idx, stream, t)
                           : ell_b<float, 2>(MP, phase_b, a, tab, val, idx, stream, t);
        case 3: return f64 ? ell_b<double, 3>(MP, phase_b, a, tab, val, idx, stream, t)
                           : ell_b<float, 3>(MP, phase_b, a, tab, val, idx, stream, t);
        case 4: return f64 ? ell_b<double, 4>(MP, phase_b, a, tab, val, idx, stream, t)
                           : ell_b<float, 4>(MP, phase_b, a, tab, val, idx, stream, t);
    }
    return hipErrorInvalidValue;
}

template <int MP>
static hipError_t invert_mp(int b, const double *diag, const int *sizes, double *blk, int L,
                            DevState *st, hipStream_t s) {
    if constexpr (MP >= 32)
        hipLaunchKernelGGL((k_invert_mfma<MP>), dim3(L), dim3(64 * inv_waves(MP)), 0, s, diag,
                           sizes, blk, 2 * b + 1, b, st);
    else
        hipLaunchKernelGGL((k_invert<MP>), dim3(L), dim3(kWG), 0, s, diag, sizes, blk, 2 * b + 1,
                           b, st);
    return hipGetLastError();
}

hipError_t launch_invert(int MP, int b, const double *diag, const int *sizes, double *blk, int L,
                         DevState *st, hipStream_t stream) {
    switch (MP) {
        case 8: return invert_mp<8>(b, diag, sizes, blk, L, st, stream);
        case 16: return invert_mp<16>(b, diag, sizes, blk, L, st, stream);
        case 32: return invert_mp<32>(b, diag, sizes, blk, L, st, stream);
        case 64: return invert_mp<64>(b, diag, sizes, blk, L, st, stream);
        case 128: return invert_mp<128>(b, diag, sizes, blk, L, st, stream);
        case 256: return invert_mp<256>(b, diag, sizes, blk, L, st, stream);
    }
    return hipErrorInvalidValue;
}

static int elementwise_groups(size_t n) {
    size_t g = (n + kWG - 1) / kWG;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_cast_blocks(const double *src, float *dst, size_t n, hipStream_t stream) {
    hipLaunchKernelGGL(k_cast, dim3(elementwise_groups(n)), dim3(kWG), 0, stream, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_widen(const float *src, double *dst, size_t n, hipStream_t stream) {
    hipLaunchKernelGGL(k_widen, dim3(elementwise_groups(n)), dim3(kWG), 0, stream, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_reset_state(DevState *st, hipStream_t stream) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, st);
    return hipGetLastError();
}

hipError_t launch_rearm(DevState *st, long long k, hipStream_t stream) {
    hipLaunchKernelGGL(k_rearm, dim3(1), dim3(64), 0, stream, st, k);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(int grid, const ChainDesc *chains, const int *range, int j,
                                 hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_finalize, dim3(grid), dim3(kWG), 0, stream, chains, range, j);
    return hipGetLastError();
}

hipError_t launch_batch_begin(int grid, const ChainDesc *chains, const int *range,
                              hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_begin, dim3((grid + kWG - 1) / kWG), dim3(kWG), 0, stream, chains,
                       range);
    return hipGetLastError();
}

hipError_t launch_batch_query(DevState *const *states, int n, QueryRow *out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_query, dim3((n + kWG - 1) / kWG), dim3(kWG), 0, stream, states, n,
                       out);
    return hipGetLastError();
}

hipError_t launch_finalize_sweep(const double *part_sum, const double *part_diff, int nslots,
                                 DevState *st, long long s, double tol, hipStream_t stream) {
    hipLaunchKernelGGL(k_finalize_sweep, dim3(1), dim3(kWG), 0, stream, part_sum, part_diff,
                       nslots, st, s, tol);
    return hipGetLastError();
}

static hipError_t reduce(const double *part, int n, int mode, DevState *st, long long slot,
                         hipStream_t stream, double tol = 0.0, double *out = nullptr) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kWG), 0, stream, part, n, mode, st, slot, tol,
                       out);
    return hipGetLastError();
}

hipError_t launch_reduce_residual(const double *part, int n, DevState *st, hipStream_t stream,
                                  double *out) {
    return reduce(part, n, kReduceResidual, st, 0, stream, 0.0, out);
}

// load/diff use at most this many groups, so their partial arrays stay small
constexpr int kAuxGroups = 1024;

hipError_t launch_load(int precision_bytes, int MP, const double *x, const long long *off,
                       const int *sizes, int L, void *w0, double *part, int nparts,
                       DevState *st, int state_slot, hipStream_t stream) {
    int groups = elementwise_groups((size_t)L * MP);
    if (groups > kAuxGroups) groups = kAuxGroups;
    if (2 * groups > nparts) groups = nparts / 2;
    if (precision_bytes == 8)
        hipLaunchKernelGGL(k_load<double>, dim3(groups), dim3(kWG), 0, stream, x, off, sizes, L,
                           MP, (double *)w0, part, state_slot);
    else
        hipLaunchKernelGGL(k_load<float>, dim3(groups), dim3(kWG), 0, stream, x, off, sizes, L,
                           MP, (float *)w0, part, state_slot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce(part, groups, kReduceLoad, st, state_slot, stream);
}

hipError_t launch_store(int precision_bytes, int MP, const void *w, const long long *off,
                        const int *sizes, int L, DevState *st, long long slot, double *x,
                        hipStream_t stream) {
    const int groups = elementwise_groups((size_t)L * MP);
    if (precision_bytes == 8)
        hipLaunchKernelGGL(k_store<double>, dim3(groups), dim3(kWG), 0, stream,
                           (const double *)w, off, sizes, L, MP, st, slot, x);
    else
        hipLaunchKernelGGL(k_store<float>, dim3(groups), dim3(kWG), 0, stream, (const float *)w,
                           off, sizes, L, MP, st, slot, x);
    return hipGetLastError();
}

template <typename T, int MP>
static hipError_t diff_mp(int rg, const void *w, const void *wp, int L, int pA, int gA, int gB,
                          const DevState *st, long long k, double *part, hipStream_t s) {
    switch (rg) {
        case 1:
            hipLaunchKernelGGL((k_diff<T, MP, 1>), dim3(gA + gB), dim3(kWG), 0, s, (const T *)w,
                               (const T *)wp, st, k, L, pA, gA, part);
            break;
        case 2:
            hipLaunchKernelGGL((k_diff<T, MP, 2>), dim3(gA + gB), dim3(kWG), 0, s, (const T *)w,
                               (const T *)wp, st, k, L, pA, gA, part);
            break;
        case 4:
            hipLaunchKernelGGL((k_diff<T, MP, 4>), dim3(gA + gB), dim3(kWG), 0, s, (const T *)w,
                               (const T *)wp, st, k, L, pA, gA, part);
            break;
        default:
            hipLaunchKernelGGL((k_diff<T, MP, 8>), dim3(gA + gB), dim3(kWG), 0, s, (const T *)w,
                               (const T *)wp, st, k, L, pA, gA, part);
    }
    return hipGetLastError();
}

hipError_t launch_diff(int precision_bytes, int MP, int variant, const void *w,
                       const void *w_prev, int L, int parity_a, DevState *st, long long k,
                       double *part, hipStream_t stream, double tol) {
    const int gA = phase_groups(precision_bytes, MP, L, parity_a, variant);
    const int gB = phase_groups(precision_bytes, MP, L, 1 - parity_a, variant);
    hipError_t e = hipErrorInvalidValue;
    if (MP > kMaxSmallMP) {
        e = launch_diff_big_partials(precision_bytes, MP, w, w_prev, parity_a, gA, gB, st, k, part,
                                     stream);
    } else if (precision_bytes == 8) {
        switch (MP) {
            case 8: e = diff_mp<double, 8>(variant_rg(8, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 16: e = diff_mp<double, 16>(variant_rg(16, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 32: e = diff_mp<double, 32>(variant_rg(32, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 64: e = diff_mp<double, 64>(variant_rg(64, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 128: e = diff_mp<double, 128>(variant_rg(128, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 256: e = diff_mp<double, 256>(variant_rg(256, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
        }
    } else {
        switch (MP) {
            case 8: e = diff_mp<float, 8>(variant_rg(8, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 16: e = diff_mp<float, 16>(variant_rg(16, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 32: e = diff_mp<float, 32>(variant_rg(32, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 64: e = diff_mp<float, 64>(variant_rg(64, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 128: e = diff_mp<float, 128>(variant_rg(128, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
            case 256: e = diff_mp<float, 256>(variant_rg(256, variant), w, w_prev, L, parity_a, gA, gB, st, k, part, stream); break;
        }
    }
    if (e != hipSuccess) return e;
    return reduce(part, gA + gB, kReduceDiff, st, k, stream, tol);
}

hipError_t launch_diff_jgs(int precision_bytes, int MP, const void *w, const void *w_prev, int L,
                           int chunks, DevState *st, long long k, double *part,
                           hipStream_t stream, double tol) {
    // the large blocks' sweep records one partial per (level, slice)
    const bool big = MP > kMaxSmallMP;
    hipError_t e = big ? launch_diff_big_levels(precision_bytes, MP, w, w_prev, L, st, k, part,
                                                stream)
                       : launch_diff_jgs_partials(precision_bytes, MP, w, w_prev, L, chunks, st, k,
                                                  part, stream);
    if (e != hipSuccess) return e;
    return reduce(part, big ? L * big_slices(precision_bytes, MP) : chunks, kReduceDiff, st, k,
                  stream, tol);
}

template <typename T, int B>
static hipError_t residual_b(int MP, const double *blk, const double *diag, const void *w,
                             int L, DevState *st, long long slot, double *part, hipStream_t s,
                             double *out) {
    const int groups = reduce_groups(MP, L);
    const T *wt = (const T *)w;
    switch (MP) {
        case 8:
            hipLaunchKernelGGL((k_residual<T, 8, B>), dim3(groups), dim3(kWG), 0, s, blk, diag,
                               wt, L, st, slot, part);
            break;
        case 16:
            hipLaunchKernelGGL((k_residual<T, 16, B>), dim3(groups), dim3(kWG), 0, s, blk, diag,
                               wt, L, st, slot, part);
            break;
        case 32:
            hipLaunchKernelGGL((k_residual<T, 32, B>), dim3(groups), dim3(kWG), 0, s, blk, diag,
                               wt, L, st, slot, part);
            break;
        case 64:
            hipLaunchKernelGGL((k_residual<T, 64, B>), dim3(groups), dim3(kWG), 0, s, blk, diag,
                               wt, L, st, slot, part);
            break;
        case 128:
            hipLaunchKernelGGL((k_residual<T, 128, B>), dim3(groups), dim3(kWG), 0, s, blk, diag,
                               wt, L, st, slot, part);
            break;
        default:
            return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return reduce(part, groups, kReduceResidual, st, 0, s, 0.0, out);
}

hipError_t launch_residual(int precision_bytes, int MP, int b, const double *blk64,
                           const double *diag64, const void *w, int L, DevState *st,
                           long long slot, double *part, hipStream_t stream, double *out) {
    const bool f64 = precision_bytes == 8;
    switch (b) {
        case 1: return f64 ? residual_b<double, 1>(MP, blk64, diag64, w, L, st, slot, part, stream, out)
                           : residual_b<float, 1>(MP, blk64, diag64, w, L, st, slot, part, stream, out);
        case 2: return f64 ? residual_b<double, 2>(MP, blk64, diag64, w, L, st, slot, part, stream, out)
                           : residual_b<float, 2>(MP, blk64, diag64, w, L, st, slot, part, stream, out);
        case 3: return f64 ? residual_b<double, 3>(MP, blk64, diag64, w, L, st, slot, part, stream, out)
                           : residual_b<float, 3>(MP, blk64, diag64, w, L, st, slot, part, stream, out);
        case 4: return f64 ? residual_b<double, 4>(MP, blk64, diag64, w, L, st, slot, part, stream, out)
                           : residual_b<float, 4>(MP, blk64, diag64, w, L, st, slot, part, stream, out);
    }
    return hipErrorInvalidValue;
}

}  // namespace stc
