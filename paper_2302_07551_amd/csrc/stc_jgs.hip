// Algorithm 1 (section 2), the paper's comparison method: one sweep of the
// block Jacobi / Gauss-Seidel splitting over p chunks of consecutive levels.
// Block Jacobi across the chunks: a level reads the previous iterate from
// every other chunk.  Block Gauss-Seidel inside a chunk: its levels are taken
// in order, each reading the fresh values of the chunk's earlier levels.
// With p = 1 this is plain block Gauss-Seidel, with p = L block Jacobi.
//
// One workgroup per chunk.  Its levels are sequential, so each level uses the
// whole workgroup (the sweep tile with 8 row groups; blocks below 64 leave
// the other teams idle), and the fresh values of the last B levels stay in
// LDS.  The sweep follows the conventions of the staircase kernels: W_s from
// W_{s-1} scaled by 1 / e^T W_{s-2}, per-chunk partial sums of e^T W_s and of
// the change of sweep s - 2, and an extra workgroup that records sweep s - 1.
#include "stc_device.h"

namespace stc {

template <typename T, int MP, int B, bool NT>
__global__ __launch_bounds__(kWG) void k_sweep_jgs(SweepLaunch a, int chunks) {
    using TL = Tile<T, MP, 8>;
    using VT = typename Vec16<T>::type;
    constexpr int NB = 2 * B + 1;
    constexpr int VEC = TL::VEC, CT = TL::CT, R = TL::R, RPT = TL::RPT, TS = TL::TS,
                  PF = TL::PF;
    constexpr size_t BS = (size_t)MP * MP;
    __shared__ T red[R * MP];
    __shared__ T rv[MP];
    __shared__ T ring[B * MP];   // fresh values of level s at ring[(s % B) MP]
    __shared__ double sh[4 * kWG / 64];
    int q = blockIdx.x;
    if (a.fold) {   // the reduction workgroup first (see k_sweep)
        if (q == 0) {
            fold_previous(a, sh);
            return;
        }
        --q;
    }
    const DevState *st = a.st;
    const int tid = threadIdx.x;
    const int team = tid / TS, tt = tid - team * TS;
    const int c = tt % CT, g = tt / CT;
    const bool worker = team == 0;
    const bool live = st->stop_flag == 0;
    const T sc = (T)st->inv_sigma[(a.s - 2) & kRingMask];
    const int k0 = jgs_first(q, a.L, chunks), k1 = jgs_first(q + 1, a.L, chunks);
    const ChainView<T> v = view_of<T>(a);
    const T *w_old = v.w_old;
    T *w_new = v.w_new;
    double i2 = 0.0, i3 = 0.0;
    if (a.s >= 3) {
        i2 = st->inv_sigma[(a.s - 2) & kRingMask];
        i3 = st->inv_sigma[(a.s - 3) & kRingMask];
    }
    double zs = 0.0, dd = 0.0;
    for (int k = k0; k < k1; ++k) {
        const T *base = v.blk + (size_t)k * NB * BS;
        const T *wb = base + (size_t)B * BS + c * VEC;
        VT acc = (VT)(T)0;
        VT vpre[PF];
        if (worker) {
#pragma unroll
            for (int d = -B; d <= B; ++d) {
                if (d == 0) continue;
                const int s = k + d;
                if (s < 0 || s >= a.L) continue;   // no block there
                // the chunk's earlier levels are fresh; everything else is old
                const bool fresh = s >= k0 && s < k;
                const T *gb = base + (size_t)(d + B) * BS + c * VEC;
#pragma unroll
                for (int qq = 0; qq < RPT; ++qq) {
                    const int row = g + R * qq;
                    const VT blkv = stream_load<VT, NT>((const VT *)(gb + (size_t)row * MP));
                    const T x = fresh ? ring[(s % B) * MP + row] : w_old[(size_t)s * MP + row] * sc;
                    acc += blkv * x;
                }
            }
            // rows of W_k fetched before the reduction, so they stream meanwhile
#pragma unroll
            for (int qq = 0; qq < PF; ++qq)
                vpre[qq] = stream_load<VT, NT>((const VT *)(wb + (size_t)(g + R * qq) * MP));
#pragma unroll
            for (int e = 0; e < VEC; ++e) red[g * MP + c * VEC + e] = acc[e];
        }
        __syncthreads();
        if (worker) {
#pragma unroll
            for (int e = tt; e < MP; e += TS) {
                T r = 0;
#pragma unroll
                for (int gg = 0; gg < R; ++gg) r += red[gg * MP + e];
                rv[e] = r;
            }
        }
        __syncthreads();
        // z_k = W_k r_k
        if (worker) {
            VT acc2 = (VT)(T)0;
#pragma unroll
            for (int qq = 0; qq < RPT; ++qq) {
                const int row = g + R * qq;
                const VT wv = (qq < PF) ? vpre[qq < PF ? qq : 0]
                                        : stream_load<VT, NT>((const VT *)(wb + (size_t)row * MP));
                acc2 += wv * rv[row];
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) red[g * MP + c * VEC + e] = acc2[e];
        }
        __syncthreads();
        if (worker) {
#pragma unroll
            for (int e = tt; e < MP; e += TS) {
                T z = 0;
#pragma unroll
                for (int gg = 0; gg < R; ++gg) z += red[gg * MP + e];
                ring[(k % B) * MP + e] = z;
                if (live) w_new[(size_t)k * MP + e] = z;
                zs += (double)z;
                if (a.s >= 3)
                    dd += fabs((double)v.w_d1[(size_t)k * MP + e] * i2 -
                               (double)v.w_d2[(size_t)k * MP + e] * i3);
            }
        }
        __syncthreads();   // the ring and red are ready for the next level
    }
    double S = zs, D = dd;
    block_sum2(S, D, sh);
    if (live && tid == 0) {
        a.part_sum[q] = S;
        a.part_diff[q] = D;
    }
}

// The change of sweep k in the JGS kernel's geometry and order (one
// workgroup per chunk, the same terms per thread and the same workgroup
// sum), so a burst's flush records what the next sweep's partials would.
template <typename T, int MP>
__global__ __launch_bounds__(kWG) void k_diff_jgs(const T *w, const T *wp, const DevState *st,
                                                   long long k, int L, int chunks, double *part) {
    using TL = Tile<T, MP, 8>;
    __shared__ double sh[4 * kWG / 64];
    const int q = blockIdx.x, tid = threadIdx.x;
    const int team = tid / TL::TS, tt = tid - team * TL::TS;
    const int k0 = jgs_first(q, L, chunks), k1 = jgs_first(q + 1, L, chunks);
    const double i2 = st->inv_sigma[k & kRingMask];
    const double i3 = st->inv_sigma[(k - 1) & kRingMask];
    double dd = 0.0;
    if (team == 0)
        for (int lev = k0; lev < k1; ++lev) {
#pragma unroll
            for (int e = tt; e < MP; e += TL::TS)
                dd += fabs((double)w[(size_t)lev * MP + e] * i2 -
                           (double)wp[(size_t)lev * MP + e] * i3);
        }
    const double D = block_sum(dd, sh);
    if (tid == 0) part[q] = D;
}

template <typename T, int MP, int B>
static hipError_t jgs_mpb(bool nt, int chunks, const SweepLaunch &a, hipStream_t s,
                          LaunchTimer t) {
    const int groups = chunks + (a.fold ? 1 : 0);
    if (nt)
        launch_timed(k_sweep_jgs<T, MP, B, true>, groups, s, t, a, chunks);
    else
        launch_timed(k_sweep_jgs<T, MP, B, false>, groups, s, t, a, chunks);
    return hipGetLastError();
}

template <typename T, int B>
static hipError_t jgs_b(int MP, bool nt, int chunks, const SweepLaunch &a, hipStream_t s,
                        LaunchTimer t) {
    switch (MP) {
        case 8: return jgs_mpb<T, 8, B>(nt, chunks, a, s, t);
        case 16: return jgs_mpb<T, 16, B>(nt, chunks, a, s, t);
        case 32: return jgs_mpb<T, 32, B>(nt, chunks, a, s, t);
        case 64: return jgs_mpb<T, 64, B>(nt, chunks, a, s, t);
        case 128: return jgs_mpb<T, 128, B>(nt, chunks, a, s, t);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t jgs_t(int MP, int b, bool nt, int chunks, const SweepLaunch &a, hipStream_t s,
                        LaunchTimer t) {
    switch (b) {
        case 1: return jgs_b<T, 1>(MP, nt, chunks, a, s, t);
        case 2: return jgs_b<T, 2>(MP, nt, chunks, a, s, t);
        case 3: return jgs_b<T, 3>(MP, nt, chunks, a, s, t);
        case 4: return jgs_b<T, 4>(MP, nt, chunks, a, s, t);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_jgs(int precision_bytes, int MP, int b, bool nt, int chunks,
                            const SweepLaunch &a, hipStream_t stream, LaunchTimer t) {
    if (chunks < 1 || chunks > a.L) return hipErrorInvalidValue;
    return precision_bytes == 8 ? jgs_t<double>(MP, b, nt, chunks, a, stream, t)
                                : jgs_t<float>(MP, b, nt, chunks, a, stream, t);
}

template <typename T, int MP>
static hipError_t diff_jgs_mp(const void *w, const void *wp, int L, int chunks,
                              const DevState *st, long long k, double *part, hipStream_t s) {
    hipLaunchKernelGGL((k_diff_jgs<T, MP>), dim3(chunks), dim3(kWG), 0, s, (const T *)w,
                       (const T *)wp, st, k, L, chunks, part);
    return hipGetLastError();
}

template <typename T>
static hipError_t diff_jgs_t(int MP, const void *w, const void *wp, int L, int chunks,
                             const DevState *st, long long k, double *part, hipStream_t s) {
    switch (MP) {
        case 8: return diff_jgs_mp<T, 8>(w, wp, L, chunks, st, k, part, s);
        case 16: return diff_jgs_mp<T, 16>(w, wp, L, chunks, st, k, part, s);
        case 32: return diff_jgs_mp<T, 32>(w, wp, L, chunks, st, k, part, s);
        case 64: return diff_jgs_mp<T, 64>(w, wp, L, chunks, st, k, part, s);
        case 128: return diff_jgs_mp<T, 128>(w, wp, L, chunks, st, k, part, s);
        case 256: return diff_jgs_mp<T, 256>(w, wp, L, chunks, st, k, part, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_diff_jgs_partials(int precision_bytes, int MP, const void *w, const void *w_prev,
                                    int L, int chunks, const DevState *st, long long k,
                                    double *part, hipStream_t stream) {
    return precision_bytes == 8 ? diff_jgs_t<double>(MP, w, w_prev, L, chunks, st, k, part, stream)
                                : diff_jgs_t<float>(MP, w, w_prev, L, chunks, st, k, part, stream);
}

}  // namespace stc
