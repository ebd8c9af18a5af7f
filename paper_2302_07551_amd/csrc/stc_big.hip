// Sweep, change and residual kernels for generators of any block pattern
// partitioned into large levels (padded block sizes 512, 1024 and 2048: the
// partitions l = 512 .. 2048 of the experiments in section 3).
//
// A level of 2048 states has a 32 MB FP64 inverse W_i.  One workgroup per
// level, as in the smaller kernels, would leave a few dozen CUs to stream a
// whole phase, each through its own memory pipeline.  Here each phase of
// Algorithm 2 is two launches instead:
//   gather: r_i = -sum_{k != i} A_{i,k} x_k for every level i of the phase,
//           into a scratch vector (workgroups of 64 columns, four lanes per
//           column splitting its ELL quads; near sources fresh in phase B,
//           far sources from the previous iterate scaled by kappa, as in the
//           smaller kernels);
//   apply:  z_i = W_i r_i by column slices of W_i (workgroups of 512 bytes of
//           every row: 64 FP64 or 128 FP32 columns), each writing its slice
//           of z_i and one partial of e^T z and of the change.
// The partials, the lagged normalisation, phase B's fold and the device
// stopping test are those of the other kernels, with one partial slot per
// (level, slice).  The change kernel of a burst's flush and the residual
// kernel use the same slices.
#include "stc_device.h"

namespace stc {

namespace {

constexpr int kGatherCols = 64;             // columns per gather workgroup
constexpr int kGatherLanes = kWG / kGatherCols;   // lanes per column
constexpr int kRowGroups = 8;               // row groups of an apply workgroup

template <typename T>
struct BigTile {
    static constexpr int VEC = 16 / (int)sizeof(T);     // elements per 16-byte load
    static constexpr int CS = (kWG / kRowGroups) * VEC;  // columns of a slice: 512 bytes
};

typedef int Int4 __attribute__((ext_vector_type(4)));

}  // namespace

int big_slices(int precision_bytes, int MP) {
    return precision_bytes == 8 ? MP / BigTile<double>::CS : MP / BigTile<float>::CS;
}

int big_residual_slices(int MP) { return MP / kGatherCols; }

// r_i for the levels parity, parity + 2, ... of one phase.  Workgroup q
// takes level parity + 2 (q / (MP / 64)) and its columns 64 (q % (MP / 64))
// onward; lane gg of a column sums the column's quads gg, gg + 4, ... (near
// and far apart, each in quad order), then lanes 0 .. 3 are added in order.
template <typename T, int MP, bool PHB, bool NT>
__global__ __launch_bounds__(kWG) void k_gather_big(SweepLaunch a, const GenEntry *tab,
                                                     const T *val, const int *idx, T *rbuf) {
    constexpr int SL = MP / kGatherCols;
    __shared__ T red[kGatherLanes * kGatherCols];
    const int tid = threadIdx.x;
    const int q = blockIdx.x;
    const int lev = q / SL, sl = q - lev * SL;
    const int i = a.parity + 2 * lev;
    const int jl = tid % kGatherCols, gg = tid / kGatherCols;
    const int j = sl * kGatherCols + jl;
    const GenEntry te = tab[i];
    const int Kqn = te.Kn >> 2, Kq = (te.Kn + te.Kf) >> 2;
    const T *w_old = (const T *)a.w_old;
    const T *srcN = PHB ? (const T *)a.w_new : w_old;
    const double kappa = a.st->inv_sigma[(a.s - 2) & kRingMask];
    using VT = typename Vec16<T>::type;
    constexpr int U = sizeof(T) == 8 ? 2 : 4;   // quads per pass (FP64 quads: twice the registers)
    T accN = 0, accF = 0;
    for (int kq0 = gg; kq0 < Kq; kq0 += kGatherLanes * U) {
        // the pass's index and value loads first, then their gathers
        Int4 r4[U];
        T v[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kq = kq0 + u * kGatherLanes;
            if (kq < Kq) {
                const size_t o = (size_t)te.off + ((size_t)kq * MP + j) * 4;
                r4[u] = stream_load<Int4, NT>((const Int4 *)(idx + o));
                if constexpr (sizeof(T) == 8) {
                    const VT v01 = stream_load<VT, NT>((const VT *)(val + o));
                    const VT v23 = stream_load<VT, NT>((const VT *)(val + o + 2));
                    v[u][0] = v01[0], v[u][1] = v01[1], v[u][2] = v23[0], v[u][3] = v23[1];
                } else {
                    const VT v4 = stream_load<VT, NT>((const VT *)(val + o));
                    v[u][0] = v4[0], v[u][1] = v4[1], v[u][2] = v4[2], v[u][3] = v4[3];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kq = kq0 + u * kGatherLanes;
            if (kq < Kq) {
                const T *src = kq < Kqn ? srcN : w_old;
                const T t = v[u][0] * src[r4[u][0]] + v[u][1] * src[r4[u][1]] +
                            v[u][2] * src[r4[u][2]] + v[u][3] * src[r4[u][3]];
                if (kq < Kqn)
                    accN += t;
                else
                    accF += t;
            }
        }
    }
    const T sc = (T)kappa;
    red[gg * kGatherCols + jl] = PHB ? accN + sc * accF : sc * (accN + accF);
    __syncthreads();
    if (tid < kGatherCols) {
        T r = 0;
#pragma unroll
        for (int x = 0; x < kGatherLanes; ++x) r += red[x * kGatherCols + tid];
        rbuf[(size_t)i * MP + j] = r;
    }
}

// z_i = W_i r_i on one column slice, and the slice's partial sums.  Thread
// (g, c) streams rows g, g + 8, ... of the slice's 16-byte column group c
// (W_i is stored gather-oriented: row `row` holds the weights of r_i[row]
// in every output column); the 8 row groups are added in order in LDS.
// Phase B with a.fold: workgroup 0 reduces and records sweep s - 1 first.
template <typename T, int MP, bool PHB, bool NT>
__global__ __launch_bounds__(kWG) void k_apply_big(SweepLaunch a, const T *rbuf) {
    using VT = typename Vec16<T>::type;
    constexpr int VEC = BigTile<T>::VEC, CS = BigTile<T>::CS, S = MP / CS;
    constexpr int RPT = MP / kRowGroups;   // rows per thread
    constexpr int PW = 16;                 // rows in flight before r_i is staged
    static_assert(RPT % PW == 0, "rows per thread in whole prefetch batches");
    __shared__ T rv[MP];
    __shared__ T red[kRowGroups * CS];
    __shared__ double sh[4 * kWG / 64];
    int q = blockIdx.x;
    if (PHB && a.fold) {
        if (q == 0) {
            fold_previous(a, sh);
            return;
        }
        --q;
    }
    const int tid = threadIdx.x;
    const int lev = q / S, sl = q - lev * S;
    const int i = a.parity + 2 * lev;
    const int c = tid % (CS / VEC), g = tid / (CS / VEC);
    const int j0 = sl * CS;
    const T *wb = (const T *)a.blk + (size_t)i * MP * MP + j0 + c * VEC;

    // the first batch of rows goes out before r_i is staged; afterwards each
    // batch is issued before the previous one is used
    VT cur[PW];
#pragma unroll
    for (int u = 0; u < PW; ++u)
        cur[u] = stream_load<VT, NT>((const VT *)(wb + (size_t)(g + kRowGroups * u) * MP));
    const T *r = rbuf + (size_t)i * MP;
#pragma unroll
    for (int u = 0; u < MP / kWG; ++u) rv[tid + u * kWG] = r[tid + u * kWG];
    __syncthreads();

    VT acc = (VT)(T)0;
    for (int q0 = 0; q0 < RPT; q0 += PW) {
        VT nxt[PW];
        if (q0 + PW < RPT) {
#pragma unroll
            for (int u = 0; u < PW; ++u)
                nxt[u] = stream_load<VT, NT>(
                    (const VT *)(wb + (size_t)(g + kRowGroups * (q0 + PW + u)) * MP));
        }
#pragma unroll
        for (int u = 0; u < PW; ++u) acc += cur[u] * rv[g + kRowGroups * (q0 + u)];
#pragma unroll
        for (int u = 0; u < PW; ++u) cur[u] = nxt[u];
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) red[g * CS + c * VEC + e] = acc[e];
    __syncthreads();

    const DevState *st = a.st;
    const bool live = st->stop_flag == 0;
    double zs = 0.0, dd = 0.0;
    if (live && tid < CS) {
        T z = 0;
#pragma unroll
        for (int x = 0; x < kRowGroups; ++x) z += red[x * CS + tid];
        const size_t e = (size_t)i * MP + j0 + tid;
        ((T *)a.w_new)[e] = z;
        zs = (double)z;
        if (a.s >= 3) {
            const double i2 = st->inv_sigma[(a.s - 2) & kRingMask];
            const double i3 = st->inv_sigma[(a.s - 3) & kRingMask];
            dd = fabs((double)((const T *)a.w_d1)[e] * i2 - (double)((const T *)a.w_d2)[e] * i3);
        }
    }
    double Ssum = zs, D = dd;
    block_sum2(Ssum, D, sh);
    if (live && tid == 0) {
        a.part_sum[a.slot0 + q] = Ssum;
        a.part_diff[a.slot0 + q] = D;
    }
}

// The change of sweep k per (level, slice), in the apply kernel's geometry
// and order (the flush's partials equal the next sweep's bit for bit).
template <typename T, int MP>
__global__ __launch_bounds__(kWG) void k_diff_big(const T *w, const T *wp, const DevState *st,
                                                   long long k, int parity_a, int groups_a,
                                                   double *part) {
    constexpr int CS = BigTile<T>::CS, S = MP / CS;
    __shared__ double sh[4 * kWG / 64];
    const int tid = threadIdx.x;
    const bool in_a = (int)blockIdx.x < groups_a;
    const int q = in_a ? blockIdx.x : blockIdx.x - groups_a;
    const int parity = in_a ? parity_a : 1 - parity_a;
    const int lev = q / S, sl = q - lev * S;
    const int i = parity + 2 * lev;
    double dd = 0.0;
    if (tid < CS) {
        const double i2 = st->inv_sigma[k & kRingMask];
        const double i3 = st->inv_sigma[(k - 1) & kRingMask];
        const size_t e = (size_t)i * MP + sl * CS + tid;
        dd = fabs((double)w[e] * i2 - (double)wp[e] * i3);
    }
    const double D = block_sum(dd, sh);
    if (tid == 0) part[blockIdx.x] = D;
}

// ||Q^T x||_1 per (level, 64-column slice), FP64: the slice of
// A_{i,i} x_i (dense diagonal block, 8 row groups) plus the slice's ELL
// entries applied to x (4 lanes per column), x = w * inv_sigma[slot]
// (slot < 0: w as given).
template <typename T, int MP>
__global__ __launch_bounds__(kWG) void k_residual_big(const double *diag, const GenEntry *tab,
                                                       const double *val, const int *idx,
                                                       const T *w, const DevState *st,
                                                       long long slot, double *part) {
    using VT = typename Vec16<double>::type;
    constexpr int SL = MP / kGatherCols, CT = kGatherCols / 2, R = kWG / CT;
    __shared__ double red[R * kGatherCols];
    __shared__ double red2[kGatherLanes * kGatherCols];
    __shared__ double sh[4 * kWG / 64];
    const int tid = threadIdx.x;
    const int i = blockIdx.x / SL, sl = blockIdx.x - i * SL;
    const int j0 = sl * kGatherCols;
    const double inv = slot < 0 ? 1.0 : st->inv_sigma[slot & kRingMask];
    const int c = tid % CT, g = tid / CT;
    const double *gb = diag + (size_t)i * MP * MP + j0 + 2 * c;
    const T *v = w + (size_t)i * MP;
    VT acc = (VT)0.0;
#pragma unroll 16
    for (int row = g; row < MP; row += R) {
        const VT bv = stream_load<VT, true>((const VT *)(gb + (size_t)row * MP));
        acc += bv * ((double)v[row] * inv);
    }
    const GenEntry te = tab[i];
    const int jl = tid % kGatherCols, gg = tid / kGatherCols;
    const int Kq = (te.Kn + te.Kf) >> 2;
    double off_diag = 0.0;
    for (int kq = gg; kq < Kq; kq += kGatherLanes) {
        const size_t o = (size_t)te.off + ((size_t)kq * MP + j0 + jl) * 4;
#pragma unroll
        for (int t = 0; t < 4; ++t) off_diag += val[o + t] * (double)w[idx[o + t]];
    }
    off_diag *= inv;
    red[g * kGatherCols + 2 * c] = acc[0];
    red[g * kGatherCols + 2 * c + 1] = acc[1];
    red2[gg * kGatherCols + jl] = off_diag;
    __syncthreads();
    double res = 0.0;
    if (tid < kGatherCols) {
        double t = 0.0;
#pragma unroll
        for (int x = 0; x < R; ++x) t += red[x * kGatherCols + tid];
#pragma unroll
        for (int x = 0; x < kGatherLanes; ++x) t += red2[x * kGatherCols + tid];
        res = fabs(t);
    }
    const double S = block_sum(res, sh);
    if (tid == 0) part[blockIdx.x] = S;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

template <typename T, int MP, bool NT>
hipError_t phase_big(bool phase_b, const SweepLaunch &a, const GenEntry *tab, const void *val,
                     const int *idx, void *rbuf, hipStream_t s, LaunchTimer t) {
    const int levels = (a.L - a.parity + 1) / 2;
    if (levels <= 0) return hipSuccess;
    const int gg = levels * (MP / kGatherCols);
    const int ga = levels * (MP / BigTile<T>::CS) + ((phase_b && a.fold) ? 1 : 0);
    // the two launches of the phase are timed as one span
    const LaunchTimer t0{t.start, nullptr}, t1{nullptr, t.stop};
    if (phase_b) {
        launch_timed(k_gather_big<T, MP, true, NT>, gg, s, t0, a, tab, (const T *)val, idx,
                     (T *)rbuf);
        launch_timed(k_apply_big<T, MP, true, NT>, ga, s, t1, a, (const T *)rbuf);
    } else {
        launch_timed(k_gather_big<T, MP, false, NT>, gg, s, t0, a, tab, (const T *)val, idx,
                     (T *)rbuf);
        launch_timed(k_apply_big<T, MP, false, NT>, ga, s, t1, a, (const T *)rbuf);
    }
    return hipGetLastError();
}

template <typename T, bool NT>
hipError_t phase_big_t(int MP, bool phase_b, const SweepLaunch &a, const GenEntry *tab,
                       const void *val, const int *idx, void *rbuf, hipStream_t s,
                       LaunchTimer t) {
    switch (MP) {
        case 512: return phase_big<T, 512, NT>(phase_b, a, tab, val, idx, rbuf, s, t);
        case 1024: return phase_big<T, 1024, NT>(phase_b, a, tab, val, idx, rbuf, s, t);
        case 2048: return phase_big<T, 2048, NT>(phase_b, a, tab, val, idx, rbuf, s, t);
    }
    return hipErrorInvalidValue;
}

template <typename T, int MP>
void diff_big(const void *w, const void *wp, int parity_a, int gA, int gB, const DevState *st,
              long long k, double *part, hipStream_t s) {
    hipLaunchKernelGGL((k_diff_big<T, MP>), dim3(gA + gB), dim3(kWG), 0, s, (const T *)w,
                       (const T *)wp, st, k, parity_a, gA, part);
}

template <typename T>
hipError_t diff_big_t(int MP, const void *w, const void *wp, int parity_a, int gA, int gB,
                      const DevState *st, long long k, double *part, hipStream_t s) {
    switch (MP) {
        case 512: diff_big<T, 512>(w, wp, parity_a, gA, gB, st, k, part, s); break;
        case 1024: diff_big<T, 1024>(w, wp, parity_a, gA, gB, st, k, part, s); break;
        case 2048: diff_big<T, 2048>(w, wp, parity_a, gA, gB, st, k, part, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int MP>
void residual_big(int groups, const double *diag, const GenEntry *tab, const double *val,
                  const int *idx, const void *w, const DevState *st, long long slot, double *part,
                  hipStream_t s) {
    hipLaunchKernelGGL((k_residual_big<T, MP>), dim3(groups), dim3(kWG), 0, s, diag, tab, val,
                       idx, (const T *)w, st, slot, part);
}

template <typename T>
hipError_t residual_big_t(int MP, int groups, const double *diag, const GenEntry *tab,
                          const double *val, const int *idx, const void *w, const DevState *st,
                          long long slot, double *part, hipStream_t s) {
    switch (MP) {
        case 512: residual_big<T, 512>(groups, diag, tab, val, idx, w, st, slot, part, s); break;
        case 1024: residual_big<T, 1024>(groups, diag, tab, val, idx, w, st, slot, part, s); break;
        case 2048: residual_big<T, 2048>(groups, diag, tab, val, idx, w, st, slot, part, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep_phase_big(int precision_bytes, int MP, bool phase_b, bool nt,
                                  const SweepLaunch &a, const GenEntry *tab, const void *val,
                                  const int *idx, void *rbuf, hipStream_t stream, LaunchTimer t) {
    if (!rbuf) return hipErrorInvalidValue;
    if (precision_bytes == 8)
        return nt ? phase_big_t<double, true>(MP, phase_b, a, tab, val, idx, rbuf, stream, t)
                  : phase_big_t<double, false>(MP, phase_b, a, tab, val, idx, rbuf, stream, t);
    return nt ? phase_big_t<float, true>(MP, phase_b, a, tab, val, idx, rbuf, stream, t)
              : phase_big_t<float, false>(MP, phase_b, a, tab, val, idx, rbuf, stream, t);
}

hipError_t launch_diff_big_partials(int precision_bytes, int MP, const void *w, const void *w_prev,
                                    int parity_a, int gA, int gB, const DevState *st, long long k,
                                    double *part, hipStream_t stream) {
    return precision_bytes == 8
               ? diff_big_t<double>(MP, w, w_prev, parity_a, gA, gB, st, k, part, stream)
               : diff_big_t<float>(MP, w, w_prev, parity_a, gA, gB, st, k, part, stream);
}

hipError_t launch_residual_big_partials(int precision_bytes, int MP, int groups,
                                        const double *diag, const GenEntry *tab, const double *val,
                                        const int *idx, const void *w, const DevState *st,
                                        long long slot, double *part, hipStream_t stream) {
    return precision_bytes == 8
               ? residual_big_t<double>(MP, groups, diag, tab, val, idx, w, st, slot, part, stream)
               : residual_big_t<float>(MP, groups, diag, tab, val, idx, w, st, slot, part, stream);
}

}  // namespace stc
