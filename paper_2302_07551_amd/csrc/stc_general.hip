// Sweep and residual kernels for generators of any block pattern.
//
// The levels of such a generator may exchange probability with any other
// level (the general localized case of section 2), so the off-diagonal part
// of a level cannot be staged as a fixed set of neighbour blocks.  Each level
// keeps its off-diagonal entries of A = Q^T as a column-major ELL (GenEntry)
// with 32-bit indices into the padded iterate, split into the near segment
// (sources in levels i - 1 and i + 1, the J_i of a stair row) and the far
// segment (all other levels).  Algorithm 2 then reads, per level i:
//   phase A (diagonal-only rows): r_i = -sum_{k != i} A_{i,k} x_k, all from the
//            previous iterate;
//   phase B (stair rows): the near segment from the fresh phase-A iterate,
//            the far segment from the previous one;
// and solves z_i = W_i r_i with the dense inverse W_i = (-A_{i,i})^{-1}.
// The normalisation, the change and the stopping test are those of the
// banded kernels (lagged scales, per-group partials, phase B's fold).
#include "stc_device.h"

namespace stc {

typedef int Int4 __attribute__((ext_vector_type(4)));

// Quads of column j of a level's ELL, U per pass: the near segment's quads
// are 0 .. Kqn-1 and the far segment's Kqn .. Kq-1 (the far segment starts
// right after the near one, so quad kq sits at off + (kq MP + j) 4 in both).
// The lanes gg0, gg0 + G, ... of the column split the quads.  load() issues
// a pass's index and value loads; use() gathers the sources and adds near
// and far terms to their own sums, each in quad order.
template <typename T, int MP, int G, int U, bool NT>
struct GenPass {
    Int4 r4[U];
    T v[U][4];

    __device__ inline void load(const T *val, const int *idx, size_t base, int Kq, int kq0, int j) {
        using VT = typename Vec16<T>::type;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kq = kq0 + u * G;
            // no default value: use() reads a quad under the same test, and a
            // merge with a default would make the loads wait right here
            if (kq < Kq) {
                const size_t o = base + ((size_t)kq * MP + j) * 4;
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
    }

    __device__ inline void use(int Kq, int Kqn, int kq0, const T *srcN, const T *srcF, T &accN,
                               T &accF) const {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kq = kq0 + u * G;
            if (kq < Kq) {
                const T *src = kq < Kqn ? srcN : srcF;
                const T t = v[u][0] * src[r4[u][0]] + v[u][1] * src[r4[u][1]] +
                            v[u][2] * src[r4[u][2]] + v[u][3] * src[r4[u][3]];
                if (kq < Kqn)
                    accN += t;
                else
                    accF += t;
            }
        }
    }
};

// One workgroup of a half-sweep: LPW levels (team t of group q owns level
// parity + 2 (q LPW + t)), then the group's partial sums into slot slot0 + q.
// NT: non-temporal loads of the stored entries (a stage whose blocks and
// entries exceed the last-level cache streams them; a smaller one keeps them
// cached from sweep to sweep).
template <typename T, int MP, bool PHB, bool NT>
__device__ inline void sweep_group_gen(const ChainView<T> &a, const GenEntry *tab, const T *val,
                                       const int *idx, int q, bool live, double inv_old,
                                       T *red_base, T *rv_base, double *sh) {
    using TL = Tile<T, MP, 8>;
    using VT = typename Vec16<T>::type;
    constexpr int VEC = TL::VEC, CT = TL::CT, R = TL::R, RPT = TL::RPT, TS = TL::TS,
                  LPW = TL::LPW, PF = TL::PF;
    constexpr int G = TS / MP;            // lanes splitting the ELL slots of a column
    constexpr size_t BS = (size_t)MP * MP;
    static_assert(G >= 1 && G <= R, "team narrower than a block");
    // With one level per workgroup (the large blocks) a CU holds few waves,
    // so the waves keep all their W_i rows in flight, not just PF of them:
    // the registers are there, and the loads in flight set the bandwidth.
    constexpr int PW = LPW == 1 ? (RPT < 32 ? RPT : 32) : PF;

    const DevState *st = a.st;
    const int tid = threadIdx.x;
    const int team = tid / TS, tt = tid - team * TS;
    const int c = tt % CT, g = tt / CT;
    T *red = red_base + team * (R * MP);
    T *rv = rv_base + team * MP;
    const int i = a.parity + 2 * (q * LPW + team);
    const bool active = i < a.L;
    // a team of whole waves has one level per wave: make it wave-uniform, so
    // its table entry comes through a scalar load and the first vector loads
    // need not wait for it behind the vector queue
    const int ic = TS >= 64 ? __builtin_amdgcn_readfirstlane(active ? i : a.parity)
                            : (active ? i : a.parity);
    T *w_new = a.w_new;
    const T *wb = a.blk + (size_t)ic * BS + c * VEC;   // W_ic, the only dense block
    const GenEntry te = tab[ic];

    // r_i[j] = sum over the column's slots of val * source.  The lane's first
    // pass of ELL loads goes out before the W_i rows: loads return in order,
    // so behind the rows the gather would wait for the whole block first.
    // quads per pass: FP64 quads hold twice the registers, so two, except
    // with one lane per column (blocks of 256), where four keep a column's
    // usual four quads in one pass (one round of index loads, one of
    // gathers); the quads are added in the same order either way
    constexpr int U = (sizeof(T) == 4 || G == 1) ? 4 : 2;
    const int j = tt % MP, gg0 = tt / MP;
    const int Kqn = te.Kn >> 2, Kq = (te.Kn + te.Kf) >> 2;
    GenPass<T, MP, G, U, NT> pass;
    pass.load(val, idx, (size_t)te.off, Kq, gg0, j);

    // rows of W_i stream while the gathers run
    VT vpre[PW];
#pragma unroll
    for (int qq = 0; qq < PW; ++qq)
        vpre[qq] = stream_load<VT, NT>((const VT *)(wb + (size_t)(g + R * qq) * MP));

    // phase B reads the near sources fresh; the previous iterate's terms are
    // scaled by kappa once, after their sum
    const T *srcN = PHB ? (const T *)w_new : a.w_old;
    T accN = 0, accF = 0;
    pass.use(Kq, Kqn, gg0, srcN, a.w_old, accN, accF);
    for (int kq0 = gg0 + G * U; kq0 < Kq; kq0 += G * U) {
        pass.load(val, idx, (size_t)te.off, Kq, kq0, j);
        pass.use(Kq, Kqn, kq0, srcN, a.w_old, accN, accF);
    }
    const T sc = (T)inv_old;
    red[gg0 * MP + j] = PHB ? accN + sc * accF : sc * (accN + accF);
    __syncthreads();
    if (tt < MP) {
        T r = 0;
#pragma unroll
        for (int x = 0; x < G; ++x) r += red[x * MP + tt];
        rv[tt] = r;
    }
    __syncthreads();

    // z_i = W_i r_i (dense)
    VT acc2 = (VT)(T)0;
#pragma unroll
    for (int qq = 0; qq < RPT; ++qq) {
        const int row = g + R * qq;
        const VT wv = (qq < PW) ? vpre[qq < PW ? qq : 0]
                                : stream_load<VT, NT>((const VT *)(wb + (size_t)row * MP));
        acc2 += wv * rv[row];
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) red[g * MP + c * VEC + e] = acc2[e];
    __syncthreads();

    double zs = 0.0, dd = 0.0;
    if (live && active && tt < MP) {
        T z = 0;
#pragma unroll
        for (int x = 0; x < R; ++x) z += red[x * MP + tt];
        w_new[(size_t)i * MP + tt] = z;
        zs = (double)z;
        if (a.s >= 3) {
            const double i2 = st->inv_sigma[(a.s - 2) & kRingMask];
            const double i3 = st->inv_sigma[(a.s - 3) & kRingMask];
            dd = fabs((double)a.w_d1[(size_t)i * MP + tt] * i2 -
                      (double)a.w_d2[(size_t)i * MP + tt] * i3);
        }
    }
    double S = zs, D = dd;
    block_sum2(S, D, sh);
    if (live && tid == 0) {
        a.part_sum[a.slot0 + q] = S;
        a.part_diff[a.slot0 + q] = D;
    }
}

template <typename T, int MP, bool PHB, bool NT>
__global__ __launch_bounds__(kWG) void k_sweep_gen(SweepLaunch a, const GenEntry *tab,
                                                    const void *val, const int *idx) {
    using TL = Tile<T, MP, 8>;
    __shared__ T red[TL::LPW * TL::R * MP];
    __shared__ T rv[TL::LPW * MP];
    __shared__ double sh[4 * kWG / 64];
    int q = blockIdx.x;
    if (PHB && a.fold) {   // the reduction workgroup first (see k_sweep)
        if (q == 0) {
            fold_previous(a, sh);
            return;
        }
        --q;
    }
    const bool live = a.st->stop_flag == 0;
    const double kappa = a.st->inv_sigma[(a.s - 2) & kRingMask];
    sweep_group_gen<T, MP, PHB, NT>(view_of<T>(a), tab, (const T *)val, idx, q, live, kappa, red,
                                    rv, sh);
}

// Algorithm 1 (JGS) on a generator of any block pattern: one workgroup per
// chunk of consecutive levels k0 .. k1 - 1, taken in order (block
// Gauss-Seidel inside the chunk, block Jacobi across chunks).  Level k's
// entries read W_s for sources in the chunk's earlier levels (written by
// this workgroup before a barrier) and the previous iterate, scaled by
// kappa, everywhere else; z_k = W_k r_k with the dense inverse.  The sums
// e^T z and the change are accumulated per thread over the chunk's levels
// in the dense JGS kernel's geometry (team 0, elements tt, tt + TS, ...),
// so its change kernel gives the flush the same partials.  The extra
// workgroup of a.fold records sweep s - 1 first.
template <typename T, int MP, bool NT>
__global__ __launch_bounds__(kWG) void k_sweep_jgs_gen(SweepLaunch a, int chunks,
                                                        const GenEntry *tab, const void *valv,
                                                        const int *idx) {
    using TL = Tile<T, MP, 8>;
    using VT = typename Vec16<T>::type;
    constexpr int VEC = TL::VEC, CT = TL::CT, R = TL::R, RPT = TL::RPT, TS = TL::TS;
    constexpr int G = TS / MP;            // lanes splitting the ELL slots of a column
    constexpr size_t BS = (size_t)MP * MP;
    __shared__ T red[R * MP];
    __shared__ T rv[MP];
    __shared__ double sh[4 * kWG / 64];
    int q = blockIdx.x;
    if (a.fold) {
        if (q == 0) {
            fold_previous(a, sh);
            return;
        }
        --q;
    }
    const T *val = (const T *)valv;
    const DevState *st = a.st;
    const int tid = threadIdx.x;
    const int team = tid / TS, tt = tid - team * TS;
    const int c = tt % CT, g = tt / CT;
    const int j = tt % MP, gg0 = tt / MP;
    const bool worker = team == 0;
    const bool live = st->stop_flag == 0;
    const T sc = (T)st->inv_sigma[(a.s - 2) & kRingMask];
    const int k0 = jgs_first(q, a.L, chunks), k1 = jgs_first(q + 1, a.L, chunks);
    const T *w_old = (const T *)a.w_old, *w_d1 = (const T *)a.w_d1, *w_d2 = (const T *)a.w_d2;
    T *w_new = (T *)a.w_new;
    double i2 = 0.0, i3 = 0.0;
    if (a.s >= 3) {
        i2 = st->inv_sigma[(a.s - 2) & kRingMask];
        i3 = st->inv_sigma[(a.s - 3) & kRingMask];
    }
    double zs = 0.0, dd = 0.0;
    for (int k = k0; k < k1; ++k) {
        const T *wb = (const T *)a.blk + (size_t)k * BS + c * VEC;
        if (worker) {
            // r_k[j]: the column's slots, fresh sources (levels k0 .. k - 1)
            // and previous-iterate sources summed apart, in slot order
            const GenEntry te = tab[k];
            const int Kq = (te.Kn + te.Kf) >> 2;
            T accF = 0, accO = 0;
            for (int kq = gg0; kq < Kq; kq += G) {
                const size_t o = (size_t)te.off + ((size_t)kq * MP + j) * 4;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int si = idx[o + t];
                    const int lev = si / MP;
                    if (lev >= k0 && lev < k)
                        accF += val[o + t] * w_new[si];
                    else
                        accO += val[o + t] * w_old[si];
                }
            }
            red[gg0 * MP + j] = accF + sc * accO;
        }
        __syncthreads();
        if (worker && tt < MP) {
            T r = 0;
#pragma unroll
            for (int x = 0; x < G; ++x) r += red[x * MP + tt];
            rv[tt] = r;
        }
        __syncthreads();
        // z_k = W_k r_k
        if (worker) {
            VT acc2 = (VT)(T)0;
#pragma unroll 8
            for (int qq = 0; qq < RPT; ++qq) {
                const int row = g + R * qq;
                acc2 += stream_load<VT, NT>((const VT *)(wb + (size_t)row * MP)) * rv[row];
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
                if (live) w_new[(size_t)k * MP + e] = z;
                zs += (double)z;
                if (a.s >= 3)
                    dd += fabs((double)w_d1[(size_t)k * MP + e] * i2 -
                               (double)w_d2[(size_t)k * MP + e] * i3);
            }
        }
        __syncthreads();   // W_s of level k is visible to the chunk's next levels
    }
    double S = zs, D = dd;
    block_sum2(S, D, sh);
    if (live && tid == 0) {
        a.part_sum[q] = S;
        a.part_diff[q] = D;
    }
}

// ||Q^T x||_1 per group of levels, FP64: (Q^T x) restricted to level i is
// A_{i,i} x_i (dense diagonal block) plus the level's ELL entries applied to
// x, with x = w * inv_sigma[slot] (slot < 0: w as given).
template <typename T, int MP>
__global__ __launch_bounds__(kWG) void k_residual_gen(const double *diag, const GenEntry *tab,
                                                       const double *val, const int *idx,
                                                       const T *w, int L, const DevState *st,
                                                       long long slot, double *part) {
    using TL = Tile<double, MP, 8>;
    using VT = typename Vec16<double>::type;
    constexpr int VEC = TL::VEC, CT = TL::CT, R = TL::R, RPT = TL::RPT, TS = TL::TS,
                  LPW = TL::LPW;
    constexpr int G = TS / MP;
    constexpr size_t BS = (size_t)MP * MP;
    __shared__ double red[LPW][R][MP];
    __shared__ double red2[LPW][G][MP];
    __shared__ double sh[4 * kWG / 64];

    const int tid = threadIdx.x;
    const int team = tid / TS, tt = tid - team * TS;
    const int c = tt % CT, g = tt / CT;
    const int i = blockIdx.x * LPW + team;
    const bool active = i < L;
    const double inv = slot < 0 ? 1.0 : st->inv_sigma[slot & kRingMask];

    VT acc = (VT)0.0;
    double off_diag = 0.0;
    if (active) {
        const double *gb = diag + (size_t)i * BS + c * VEC;
        const T *v = w + (size_t)i * MP;
        // unrolled 32 rows at a time (blocks of 256 stream 128 rows per
        // thread; unrolled whole they would spill); the sum's order is the same
        constexpr int UR = RPT > 32 ? 32 : RPT;
#pragma unroll UR
        for (int qq = 0; qq < RPT; ++qq) {
            const int row = g + R * qq;
            const VT bv = stream_load<VT, true>((const VT *)(gb + (size_t)row * MP));
            acc += bv * ((double)v[row] * inv);
        }
        const GenEntry te = tab[i];
        const int j = tt % MP, gg0 = tt / MP;
        const int Kq = (te.Kn + te.Kf) >> 2;   // both segments, one source
        for (int kq = gg0; kq < Kq; kq += G) {
            const size_t o = (size_t)te.off + ((size_t)kq * MP + j) * 4;
#pragma unroll
            for (int t = 0; t < 4; ++t) off_diag += val[o + t] * (double)w[idx[o + t]];
        }
        off_diag *= inv;
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) red[team][g][c * VEC + e] = acc[e];
    red2[team][tt / MP][tt % MP] = off_diag;
    __syncthreads();
    double r = 0.0;
    if (active && tt < MP) {
        double t = 0.0;
#pragma unroll
        for (int gg = 0; gg < R; ++gg) t += red[team][gg][tt];
#pragma unroll
        for (int x = 0; x < G; ++x) t += red2[team][x][tt];
        r = fabs(t);
    }
    const double S = block_sum(r, sh);
    if (tid == 0) part[blockIdx.x] = S;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int MP, bool NT>
static hipError_t gen_mp(bool phase_b, const SweepLaunch &a, const GenEntry *tab, const void *val,
                         const int *idx, hipStream_t s, LaunchTimer t) {
    const int groups = phase_groups((int)sizeof(T), MP, a.L, a.parity, kEllGeometry) +
                       ((phase_b && a.fold) ? 1 : 0);   // + the reduction workgroup
    if (groups <= 0) return hipSuccess;
    if (phase_b)
        launch_timed(k_sweep_gen<T, MP, true, NT>, groups, s, t, a, tab, val, idx);
    else
        launch_timed(k_sweep_gen<T, MP, false, NT>, groups, s, t, a, tab, val, idx);
    return hipGetLastError();
}

template <typename T, bool NT>
static hipError_t gen_t(int MP, bool phase_b, const SweepLaunch &a, const GenEntry *tab,
                        const void *val, const int *idx, hipStream_t s, LaunchTimer t) {
    switch (MP) {
        case 8: return gen_mp<T, 8, NT>(phase_b, a, tab, val, idx, s, t);
        case 16: return gen_mp<T, 16, NT>(phase_b, a, tab, val, idx, s, t);
        case 32: return gen_mp<T, 32, NT>(phase_b, a, tab, val, idx, s, t);
        case 64: return gen_mp<T, 64, NT>(phase_b, a, tab, val, idx, s, t);
        case 128: return gen_mp<T, 128, NT>(phase_b, a, tab, val, idx, s, t);
        case 256: return gen_mp<T, 256, NT>(phase_b, a, tab, val, idx, s, t);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_phase_gen(int precision_bytes, int MP, bool phase_b, bool nt,
                                  const SweepLaunch &a, const GenEntry *tab, const void *val,
                                  const int *idx, void *rbuf, hipStream_t stream, LaunchTimer t) {
    if (MP > kMaxSmallMP)
        return launch_sweep_phase_big(precision_bytes, MP, phase_b, nt, a, tab, val, idx, rbuf,
                                      stream, t);
    if (precision_bytes == 8)
        return nt ? gen_t<double, true>(MP, phase_b, a, tab, val, idx, stream, t)
                  : gen_t<double, false>(MP, phase_b, a, tab, val, idx, stream, t);
    return nt ? gen_t<float, true>(MP, phase_b, a, tab, val, idx, stream, t)
              : gen_t<float, false>(MP, phase_b, a, tab, val, idx, stream, t);
}

template <typename T, int MP>
static void residual_gen_mp(int groups, const double *diag, const GenEntry *tab, const double *val,
                            const int *idx, const void *w, int L, const DevState *st,
                            long long slot, double *part, hipStream_t s) {
    hipLaunchKernelGGL((k_residual_gen<T, MP>), dim3(groups), dim3(kWG), 0, s, diag, tab, val, idx,
                       (const T *)w, L, st, slot, part);
}

template <typename T>
static hipError_t residual_gen_t(int MP, int groups, const double *diag, const GenEntry *tab,
                                 const double *val, const int *idx, const void *w, int L,
                                 const DevState *st, long long slot, double *part,
                                 hipStream_t s) {
    switch (MP) {
        case 8: residual_gen_mp<T, 8>(groups, diag, tab, val, idx, w, L, st, slot, part, s); break;
        case 16: residual_gen_mp<T, 16>(groups, diag, tab, val, idx, w, L, st, slot, part, s); break;
        case 32: residual_gen_mp<T, 32>(groups, diag, tab, val, idx, w, L, st, slot, part, s); break;
        case 64: residual_gen_mp<T, 64>(groups, diag, tab, val, idx, w, L, st, slot, part, s); break;
        case 128: residual_gen_mp<T, 128>(groups, diag, tab, val, idx, w, L, st, slot, part, s); break;
        case 256: residual_gen_mp<T, 256>(groups, diag, tab, val, idx, w, L, st, slot, part, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_residual_gen(int precision_bytes, int MP, const double *diag64,
                               const GenEntry *tab, const double *val64, const int *idx,
                               const void *w, int L, DevState *st, long long slot, double *part,
                               hipStream_t stream, double *out) {
    const int groups = reduce_groups(MP, L);
    const hipError_t e =
        MP > kMaxSmallMP
            ? launch_residual_big_partials(precision_bytes, MP, groups, diag64, tab, val64, idx, w,
                                           st, slot, part, stream)
        : precision_bytes == 8
            ? residual_gen_t<double>(MP, groups, diag64, tab, val64, idx, w, L, st, slot, part, stream)
            : residual_gen_t<float>(MP, groups, diag64, tab, val64, idx, w, L, st, slot, part, stream);
    if (e != hipSuccess) return e;
    return launch_reduce_residual(part, groups, st, stream, out);
}


template <typename T, int MP>
static hipError_t jgs_gen_mp(bool nt, int chunks, const SweepLaunch &a, const GenEntry *tab,
                             const void *val, const int *idx, hipStream_t s, LaunchTimer t) {
    const int groups = chunks + (a.fold ? 1 : 0);
    if (nt)
        launch_timed(k_sweep_jgs_gen<T, MP, true>, groups, s, t, a, chunks, tab, val, idx);
    else
        launch_timed(k_sweep_jgs_gen<T, MP, false>, groups, s, t, a, chunks, tab, val, idx);
    return hipGetLastError();
}

template <typename T>
static hipError_t jgs_gen_t(int MP, bool nt, int chunks, const SweepLaunch &a,
                            const GenEntry *tab, const void *val, const int *idx, hipStream_t s,
                            LaunchTimer t) {
    switch (MP) {
        case 8: return jgs_gen_mp<T, 8>(nt, chunks, a, tab, val, idx, s, t);
        case 16: return jgs_gen_mp<T, 16>(nt, chunks, a, tab, val, idx, s, t);
        case 32: return jgs_gen_mp<T, 32>(nt, chunks, a, tab, val, idx, s, t);
        case 64: return jgs_gen_mp<T, 64>(nt, chunks, a, tab, val, idx, s, t);
        case 128: return jgs_gen_mp<T, 128>(nt, chunks, a, tab, val, idx, s, t);
        case 256: return jgs_gen_mp<T, 256>(nt, chunks, a, tab, val, idx, s, t);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_jgs_gen(int precision_bytes, int MP, bool nt, int chunks,
                                const SweepLaunch &a, const GenEntry *tab, const void *val,
                                const int *idx, hipStream_t stream, LaunchTimer t) {
    if (chunks < 1 || chunks > a.L) return hipErrorInvalidValue;
    return precision_bytes == 8 ? jgs_gen_t<double>(MP, nt, chunks, a, tab, val, idx, stream, t)
                                : jgs_gen_t<float>(MP, nt, chunks, a, tab, val, idx, stream, t);
}

}  // namespace stc
