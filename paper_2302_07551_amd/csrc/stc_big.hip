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
//   apply:  z_i = W_i r_i by column slices of W_i (workgroups of 64 columns
//           of every row), each writing its slice of z_i and one partial of
//           e^T z and of the change.
// The partials, the lagged normalisation, phase B's fold and the device
// stopping test are those of the other kernels, with one partial slot per
// (level, slice).  The change kernel of a burst's flush and the residual
// kernel use the same slices.
#include "stc_device.h"

namespace stc {

namespace {

constexpr int kGatherCols = 64;             // columns per gather workgroup
constexpr int kGatherLanes = kWG / kGatherCols;   // lanes per column
constexpr int kTileDim = 64;                // tiles of the stored inverses
constexpr int kSliceCols = kTileDim;        // columns per apply workgroup
constexpr int kJgsSplit = 8;                // row ranges of a split Algorithm 1 apply
constexpr int kJgsSplitBelow = 128;         // split steps with fewer (level, slice) groups

// The inverses W_i of these blocks are stored tile-major: tile (ib, jb)
// (64 x 64, row-major inside) of a level sits at element offset
// (ib MP / 64 + jb) 4096 of the level's block.  A 64-column slice is then
// MP / 64 contiguous 32 KB tiles: streamed 5.6 % faster than 512-byte row
// segments at the block's row stride (7.06 against 6.69 TB/s, a read-only
// probe of the apply's access pattern), and the inverse's tiles are
// contiguous too.
template <int MP>
__device__ inline size_t tile_off(int ib, int jb) {
    return ((size_t)ib * (MP / kTileDim) + jb) * (kTileDim * kTileDim);
}
// Offset of row `row` of a column tile (the tile row and the row inside it).
template <int MP>
__device__ inline size_t slice_row_off(int row) {
    return (size_t)(row / kTileDim) * (MP / kTileDim) * (kTileDim * kTileDim) +
           (size_t)(row % kTileDim) * kTileDim;
}

// Apply geometry: TPR lanes cover a slice's row with 16-byte loads, R row
// groups split the rows (FP64: 32 lanes, 8 groups; FP32: 16 lanes, 16 groups).
template <typename T>
struct BigTile {
    static constexpr int VEC = 16 / (int)sizeof(T);   // elements per 16-byte load
    static constexpr int CS = kSliceCols;
    static constexpr int TPR = CS / VEC;
    static constexpr int R = kWG / TPR;
};

typedef int Int4 __attribute__((ext_vector_type(4)));

}  // namespace

int big_slices(int, int MP) { return MP / kSliceCols; }

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

// z_i = W_i r_i on one column slice (column tile sl of W_i), and the
// slice's partial sums.  Thread (g, c) streams rows g, g + R, ... of the
// slice's 16-byte column group c (W_i is stored gather-oriented: row `row`
// holds the weights of r_i[row] in every output column); the R row groups
// are added in order in LDS.
// A phase of Algorithm 2 (JGS = false): workgroup q takes level
// parity + 2 (q / (MP / 64)) and slice q % (MP / 64), slot slot0 + q; phase
// B with a.fold: workgroup 0 reduces and records sweep s - 1 first.
// A step of Algorithm 1 (JGS = true, below): level jgs_first(c) + t of chunk
// c = q / (MP / 64), slot i (MP / 64) + slice; a.fold on the first step.
// With RS > 1 (Algorithm 1 steps with few levels) workgroup q takes row
// range q % RS of (chunk, slice) q / RS, MP / RS rows, and writes its part
// of z_i to zpart (RS vectors of L MP); k_combine_big_jgs adds the parts.
template <typename T, int MP, bool PHB, bool NT, bool JGS, int RS>
__global__ __launch_bounds__(kWG) void k_apply_big(SweepLaunch a, const T *rbuf, int chunks,
                                                    int t, T *zpart) {
    using VT = typename Vec16<T>::type;
    constexpr int VEC = BigTile<T>::VEC, CS = BigTile<T>::CS, S = MP / CS;
    constexpr int TPR = BigTile<T>::TPR, R = BigTile<T>::R;
    constexpr int RPT = MP / R / RS;   // rows per thread
    constexpr int PW = 8;         // rows per batch; two batches in flight
    static_assert(RPT % PW == 0, "rows per thread in whole batches");
    __shared__ T rv[MP];
    __shared__ T red[R * CS];
    __shared__ double sh[4 * kWG / 64];
    int q = blockIdx.x;
    if ((PHB || JGS) && a.fold) {
        if (q == 0) {
            fold_previous(a, sh);
            return;
        }
        --q;
    }
    const int tid = threadIdx.x;
    int i, sl, slot, rb = 0;
    if constexpr (JGS) {
        const int cs = q / RS;
        rb = (q - cs * RS) * (MP / RS);   // first row of the range
        const int cq = cs / S;
        sl = cs - cq * S;
        i = jgs_first(cq, a.L, chunks) + t;
        if (i >= jgs_first(cq + 1, a.L, chunks)) return;   // the chunk has no level here
        slot = i * S + sl;
    } else {
        const int lev = q / S;
        sl = q - lev * S;
        i = a.parity + 2 * lev;
        slot = a.slot0 + q;
    }
    const int c = tid % TPR, g = tid / TPR;
    const int j0 = sl * CS;
    const T *wb = (const T *)a.blk + (size_t)i * MP * MP + tile_off<MP>(0, sl) + c * VEC;

    // the first batch of rows goes out before r_i is staged; afterwards each
    // batch is issued before the previous one is used
    VT cur[PW];
#pragma unroll
    for (int u = 0; u < PW; ++u)
        cur[u] = stream_load<VT, NT>((const VT *)(wb + slice_row_off<MP>(rb + g + R * u)));
    const T *r = rbuf + (size_t)i * MP;
#pragma unroll
    for (int u = 0; u < MP / kWG; ++u) rv[tid + u * kWG] = r[tid + u * kWG];
    __syncthreads();

    VT acc = (VT)(T)0;
    int q0 = 0;
    for (; q0 + PW < RPT; q0 += PW) {
        VT nxt[PW];
#pragma unroll
        for (int u = 0; u < PW; ++u)
            nxt[u] = stream_load<VT, NT>(
                (const VT *)(wb + slice_row_off<MP>(rb + g + R * (q0 + PW + u))));
#pragma unroll
        for (int u = 0; u < PW; ++u) acc += cur[u] * rv[rb + g + R * (q0 + u)];
#pragma unroll
        for (int u = 0; u < PW; ++u) cur[u] = nxt[u];
    }
#pragma unroll
    for (int u = 0; u < PW; ++u) acc += cur[u] * rv[rb + g + R * (q0 + u)];
#pragma unroll
    for (int e = 0; e < VEC; ++e) red[g * CS + c * VEC + e] = acc[e];
    __syncthreads();
    if constexpr (RS > 1) {   // this row range's part of z_i
        if (tid < CS) {
            T z = 0;
#pragma unroll
            for (int x = 0; x < R; ++x) z += red[x * CS + tid];
            zpart[(size_t)(rb / (MP / RS)) * a.L * MP + (size_t)i * MP + j0 + tid] = z;
        }
        return;
    }

    const DevState *st = a.st;
    const bool live = st->stop_flag == 0;
    double zs = 0.0, dd = 0.0;
    if (live && tid < CS) {
        T z = 0;
#pragma unroll
        for (int x = 0; x < R; ++x) z += red[x * CS + tid];
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
        a.part_sum[slot] = Ssum;
        a.part_diff[slot] = D;
    }
}

// Algorithm 1 (JGS) on the large blocks: a sweep is ceil(L / chunks) steps,
// step t taking level jgs_first(c) + t of every chunk c that has one (block
// Gauss-Seidel inside a chunk needs its levels in order; block Jacobi across
// the chunks lets a step take one level of each).  Per step a gather launch
// and an apply launch, as for a phase of Algorithm 2.  A source is fresh
// (this sweep's W_s) when its level is one of the chunk's earlier levels,
// which earlier steps wrote, and the previous iterate, scaled by kappa,
// otherwise; fresh and old terms are summed apart, each in quad order.
// Level i's slice sl records its partials in slot i (MP / 64) + sl, the
// order of k_diff_big with lstep = 1.
template <typename T, int MP, bool NT>
__global__ __launch_bounds__(kWG) void k_gather_big_jgs(SweepLaunch a, int chunks, int t,
                                                         const GenEntry *tab, const T *val,
                                                         const int *idx, T *rbuf) {
    constexpr int SL = MP / kGatherCols;
    __shared__ T red[kGatherLanes * kGatherCols];
    const int tid = threadIdx.x;
    const int q = blockIdx.x;
    const int cq = q / SL, sl = q - cq * SL;
    const int k0 = jgs_first(cq, a.L, chunks), k1 = jgs_first(cq + 1, a.L, chunks);
    const int i = k0 + t;
    if (i >= k1) return;   // the chunk has no level at this step
    const int jl = tid % kGatherCols, gg = tid / kGatherCols;
    const int j = sl * kGatherCols + jl;
    const GenEntry te = tab[i];
    const int Kq = (te.Kn + te.Kf) >> 2;
    const T *w_old = (const T *)a.w_old;
    const T *w_new = (const T *)a.w_new;
    const double kappa = a.st->inv_sigma[(a.s - 2) & kRingMask];
    using VT = typename Vec16<T>::type;
    constexpr int U = sizeof(T) == 8 ? 2 : 4;
    // fresh sources: indices k0 MP .. i MP - 1 of the padded iterate
    const unsigned lo = (unsigned)k0 * MP, span = (unsigned)(i - k0) * MP;
    T accF = 0, accO = 0;
    for (int kq0 = gg; kq0 < Kq; kq0 += kGatherLanes * U) {
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
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int si = r4[u][e];
                    if ((unsigned)si - lo < span)
                        accF += v[u][e] * w_new[si];
                    else
                        accO += v[u][e] * w_old[si];
                }
            }
        }
    }
    red[gg * kGatherCols + jl] = accF + (T)kappa * accO;
    __syncthreads();
    if (tid < kGatherCols) {
        T r = 0;
#pragma unroll
        for (int x = 0; x < kGatherLanes; ++x) r += red[x * kGatherCols + tid];
        rbuf[(size_t)i * MP + j] = r;
    }
}

// z_i of an Algorithm 1 step split over RS row ranges: the parts added in
// range order, then the slice's partial sums as k_apply_big writes them
// (slot i (MP / 64) + slice); with a.fold workgroup 0 first records sweep
// s - 1.
template <typename T, int MP, int RS>
__global__ __launch_bounds__(kWG) void k_combine_big_jgs(SweepLaunch a, int chunks, int t,
                                                          const T *zpart) {
    constexpr int CS = BigTile<T>::CS, S = MP / CS;
    __shared__ double sh[4 * kWG / 64];
    int q = blockIdx.x;
    if (a.fold) {
        if (q == 0) {
            fold_previous(a, sh);
            return;
        }
        --q;
    }
    const int cq = q / S, sl = q - cq * S;
    const int i = jgs_first(cq, a.L, chunks) + t;
    if (i >= jgs_first(cq + 1, a.L, chunks)) return;
    const int tid = threadIdx.x;
    const DevState *st = a.st;
    const bool live = st->stop_flag == 0;
    double zs = 0.0, dd = 0.0;
    if (live && tid < CS) {
        const size_t e = (size_t)i * MP + sl * CS + tid;
        T z = 0;
#pragma unroll
        for (int x = 0; x < RS; ++x) z += zpart[(size_t)x * a.L * MP + e];
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
        a.part_sum[i * S + sl] = Ssum;
        a.part_diff[i * S + sl] = D;
    }
}

// The change of sweep k per (level, slice), in the apply kernel's geometry
// and order (the flush's partials equal the next sweep's bit for bit).
// lstep = 2: the stair phases' order (phase A's levels, then phase B's);
// lstep = 1: every level in order, Algorithm 1's slots.
template <typename T, int MP>
__global__ __launch_bounds__(kWG) void k_diff_big(const T *w, const T *wp, const DevState *st,
                                                   long long k, int parity_a, int groups_a,
                                                   int lstep, double *part) {
    constexpr int CS = BigTile<T>::CS, S = MP / CS;
    __shared__ double sh[4 * kWG / 64];
    const int tid = threadIdx.x;
    const bool in_a = (int)blockIdx.x < groups_a;
    const int q = in_a ? blockIdx.x : blockIdx.x - groups_a;
    const int parity = in_a ? parity_a : 1 - parity_a;
    const int lev = q / S, sl = q - lev * S;
    const int i = parity + lstep * lev;
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
// W_i = (-Q_ii)^{-1} for the large blocks: the blocked Gauss-Jordan
// elimination of k_invert_mfma with 64-wide panels, each step spread over
// many workgroups per level instead of one.  Per panel k:
//   panel: D^{-1} = (A[k, k])^{-1}, the 64 x 64 diagonal tile inverted in LDS
//          by the same elimination (one workgroup per level), into scratch;
//   row:   A[k, j] = D^{-1} A[k, j]                 for every tile j != k;
//   trail: A[i, j] -= A[i, k] A[k, j]               for i, j != k;
//   col:   A[i, k] = -A[i, k] D^{-1}, A[k, k] = D^{-1}.
// Each launch reads only tiles that it does not write, or its own tile,
// staged in LDS before it is written back.  Tile products are 64 x 64 x 64
// on v_mfma_f64_16x16x4f64 (wave w: rows 16 w .. 16 w + 15, four 16-column
// output tiles).  No pivoting, for the reason given at k_invert; a panel
// pivot not clearly positive against the original diagonal marks the level.
// ---------------------------------------------------------------------------
namespace {

constexpr int kPanel = kTileDim;
constexpr int kPL = kPanel + 2;   // LDS row stride of a staged tile (doubles)
typedef double D2 __attribute__((ext_vector_type(2)));

// The 64 x 64 tile at g (row stride ld) into LDS t (stride kPL), by the
// workgroup's NTH threads; all loads of a thread are issued before its stores.
template <int NTH>
__device__ inline void stage_tile(const double *g, size_t ld, double *t) {
    constexpr int PER = kPanel * kPanel / 2 / NTH;
    D2 v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int p = threadIdx.x + u * NTH;
        v[u] = *(const D2 *)(g + (size_t)(p >> 5) * ld + (p & 31) * 2);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int p = threadIdx.x + u * NTH;
        t[(p >> 5) * kPL + (p & 31) * 2] = v[u][0];
        t[(p >> 5) * kPL + (p & 31) * 2 + 1] = v[u][1];
    }
}

// acc[cb] += (sa A[16 w .. 16 w + 15, :]) B[:, 16 cb .. 16 cb + 15], k = 0 .. 63
// in order (sa = 1 or -1, an exact sign).
__device__ inline void tile_mma(const double *A, const double *B, double sa, d4_t (&acc)[4]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int s4 = 0; s4 < kPanel / 4; ++s4) {
        const double av = sa * A[(16 * w + lr) * kPL + 4 * s4 + lq];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
            acc[cb] = mfma16x16x4(av, B[(4 * s4 + lq) * kPL + 16 * cb + lr], acc[cb]);
    }
}

// acc[cb][v] is element (16 w + lq + 4 v, 16 cb + lr) of a 64 x 64 tile.
__device__ inline void load_acc(const double *g, size_t ld, d4_t (&acc)[4]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[cb][v] = g[(size_t)(16 * w + lq + 4 * v) * ld + 16 * cb + lr];
}

__device__ inline void store_acc(double *g, size_t ld, const d4_t (&acc)[4]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) g[(size_t)(16 * w + lq + 4 * v) * ld + 16 * cb + lr] = acc[cb][v];
}

}  // namespace

// Row and column in the level's block of element t of its tile-major storage.
template <int MP>
__device__ inline void tile_rc(size_t t, int &r, int &c) {
    constexpr int NT = MP / kTileDim, TS = kTileDim * kTileDim;
    const int tile = (int)(t / TS), w = (int)(t % TS);
    r = (tile / NT) * kTileDim + w / kTileDim;
    c = (tile % NT) * kTileDim + w % kTileDim;
}

// W_i = -Q_ii (Q_ii row-major, W_i tile-major) on the level's states and the
// identity on its padding; the original diagonal of W_i into dorig; the
// level flags cleared.
template <int MP>
__global__ __launch_bounds__(kWG) void k_binv_init(const double *diag, const int *sizes,
                                                    double *W, double *dorig, int *bad, int L) {
    constexpr size_t BS = (size_t)MP * MP;
    const size_t n2 = (size_t)L * BS / 2;
    for (size_t p = blockIdx.x * (size_t)kWG + threadIdx.x; p < n2; p += (size_t)gridDim.x * kWG) {
        const size_t e = 2 * p;
        const int i = (int)(e / BS);
        int r, c;
        tile_rc<MP>(e - (size_t)i * BS, r, c);
        const int n = sizes[i];
        const D2 q = *(const D2 *)(diag + (size_t)i * BS + (size_t)r * MP + c);
        D2 v;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int cc = c + t;
            v[t] = (r < n && cc < n) ? -q[t] : (r == cc ? 1.0 : 0.0);
            if (r == cc) dorig[(size_t)i * MP + r] = v[t];
        }
        *(D2 *)(W + e) = v;
    }
    const size_t g = blockIdx.x * (size_t)kWG + threadIdx.x;
    if (g < (size_t)L) bad[g] = 0;
}

// The inverse of the diagonal tile (kb, kb) of every level, into dinv.
template <int MP>
__global__ __launch_bounds__(64 * inv_waves(kPanel)) void k_binv_panel(const double *W,
                                                                        const double *dorig,
                                                                        double *dinv, int *bad,
                                                                        int kb) {
    constexpr int NTH = 64 * inv_waves(kPanel);
    __shared__ double a[kPanel * kPL];
    __shared__ double dl[2][16 * 17];
    __shared__ double dor[kPanel];
    __shared__ int badl;
    const int i = blockIdx.x;
    const double *Wi = W + (size_t)i * MP * MP;
    stage_tile<NTH>(Wi + tile_off<MP>(kb, kb), kPanel, a);
    if (threadIdx.x < kPanel) dor[threadIdx.x] = dorig[(size_t)i * MP + kb * kPanel + threadIdx.x];
    if (threadIdx.x == 0) badl = 0;
    __syncthreads();
    gj_blocked<kPanel, inv_waves(kPanel), kPL>(a, dor, dl, &badl);
    __syncthreads();
    double *d = dinv + (size_t)i * kPanel * kPanel;
    for (int e = threadIdx.x; e < kPanel * kPanel; e += NTH) d[e] = a[(e / kPanel) * kPL + e % kPanel];
    if (threadIdx.x == 0 && badl) bad[i] = 1;
}

// Row panel: A[kb, jb] = D^{-1} A[kb, jb] for jb != kb.
template <int MP>
__global__ __launch_bounds__(kWG) void k_binv_row(double *W, const double *dinv, int kb) {
    constexpr int NT = MP / kPanel;
    __shared__ double D[kPanel * kPL];
    __shared__ double B[kPanel * kPL];
    const int i = blockIdx.x / (NT - 1), jj = blockIdx.x - i * (NT - 1);
    const int jb = jj + (jj >= kb);
    double *t = W + (size_t)i * MP * MP + tile_off<MP>(kb, jb);
    stage_tile<kWG>(dinv + (size_t)i * kPanel * kPanel, kPanel, D);
    stage_tile<kWG>(t, kPanel, B);
    __syncthreads();
    d4_t acc[4] = {};
    tile_mma(D, B, 1.0, acc);
    store_acc(t, kPanel, acc);
}

// Trailing update: A[ib, jb] -= A[ib, kb] A[kb, jb] for ib, jb != kb (the
// row panel already holds D^{-1} A[kb, jb]).
template <int MP>
__global__ __launch_bounds__(kWG) void k_binv_trail(double *W, int kb) {
    constexpr int NT = MP / kPanel;
    constexpr int NR = (NT - 1) * (NT - 1);
    __shared__ double C[kPanel * kPL];
    __shared__ double R[kPanel * kPL];
    const int i = blockIdx.x / NR, u = blockIdx.x - i * NR;
    const int ii = u / (NT - 1), jj = u - ii * (NT - 1);
    const int ib = ii + (ii >= kb), jb = jj + (jj >= kb);
    double *Wi = W + (size_t)i * MP * MP;
    double *t = Wi + tile_off<MP>(ib, jb);
    d4_t acc[4];
    load_acc(t, kPanel, acc);
    stage_tile<kWG>(Wi + tile_off<MP>(ib, kb), kPanel, C);
    stage_tile<kWG>(Wi + tile_off<MP>(kb, jb), kPanel, R);
    __syncthreads();
    tile_mma(C, R, -1.0, acc);
    store_acc(t, kPanel, acc);
}

// Column panel: A[ib, kb] = -A[ib, kb] D^{-1} for ib != kb; A[kb, kb] = D^{-1}.
template <int MP>
__global__ __launch_bounds__(kWG) void k_binv_col(double *W, const double *dinv, int kb) {
    constexpr int NT = MP / kPanel;
    __shared__ double C[kPanel * kPL];
    __shared__ double D[kPanel * kPL];
    const int i = blockIdx.x / NT, ib = blockIdx.x - i * NT;
    double *t = W + (size_t)i * MP * MP + tile_off<MP>(ib, kb);
    const double *d = dinv + (size_t)i * kPanel * kPanel;
    if (ib == kb) {
        for (int e = threadIdx.x; e < kPanel * kPanel; e += kWG) t[e] = d[e];
        return;
    }
    stage_tile<kWG>(t, kPanel, C);
    stage_tile<kWG>(d, kPanel, D);
    __syncthreads();
    d4_t acc[4] = {};
    tile_mma(C, D, -1.0, acc);
    store_acc(t, kPanel, acc);
}

// Padding rows and columns written as zeros; each marked level counted once.
template <int MP>
__global__ __launch_bounds__(kWG) void k_binv_final(double *W, const int *sizes, const int *bad,
                                                     DevState *st, int L) {
    constexpr size_t BS = (size_t)MP * MP;
    const size_t n = (size_t)L * BS;
    for (size_t e = blockIdx.x * (size_t)kWG + threadIdx.x; e < n; e += (size_t)gridDim.x * kWG) {
        const int i = (int)(e / BS);
        const int ni = sizes[i];
        if (ni == MP) {
            // a full level has no padding: skip to the next level
            const size_t next = (size_t)(i + 1) * BS;
            const size_t stride = (size_t)gridDim.x * kWG;
            if (next > e) e += (next - e - 1) / stride * stride;
            continue;
        }
        int r, c;
        tile_rc<MP>(e - (size_t)i * BS, r, c);
        if (!(r < ni && c < ni)) W[e] = 0.0;
    }
    const size_t g = blockIdx.x * (size_t)kWG + threadIdx.x;
    if (g < (size_t)L && bad[g]) atomicAdd(&st->bad_blocks, 1);
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
        launch_timed(k_apply_big<T, MP, true, NT, false, 1>, ga, s, t1, a, (const T *)rbuf, 0, 0,
                     (T *)nullptr);
    } else {
        launch_timed(k_gather_big<T, MP, false, NT>, gg, s, t0, a, tab, (const T *)val, idx,
                     (T *)rbuf);
        launch_timed(k_apply_big<T, MP, false, NT, false, 1>, ga, s, t1, a, (const T *)rbuf, 0,
                     0, (T *)nullptr);
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
void diff_big(const void *w, const void *wp, int parity_a, int gA, int gB, int lstep,
              const DevState *st, long long k, double *part, hipStream_t s) {
    hipLaunchKernelGGL((k_diff_big<T, MP>), dim3(gA + gB), dim3(kWG), 0, s, (const T *)w,
                       (const T *)wp, st, k, parity_a, gA, lstep, part);
}

template <typename T>
hipError_t diff_big_t(int MP, const void *w, const void *wp, int parity_a, int gA, int gB,
                      int lstep, const DevState *st, long long k, double *part, hipStream_t s) {
    switch (MP) {
        case 512: diff_big<T, 512>(w, wp, parity_a, gA, gB, lstep, st, k, part, s); break;
        case 1024: diff_big<T, 1024>(w, wp, parity_a, gA, gB, lstep, st, k, part, s); break;
        case 2048: diff_big<T, 2048>(w, wp, parity_a, gA, gB, lstep, st, k, part, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Row ranges of a split Algorithm 1 apply: at most 8, each thread keeping
// whole batches of rows (MP / (R RS) >= 8).
template <typename T, int MP>
constexpr int jgs_split() {
    return MP / (BigTile<T>::R * 8) < kJgsSplit ? MP / (BigTile<T>::R * 8) : kJgsSplit;
}

template <typename T, int MP, bool NT>
hipError_t jgs_big(int chunks, const SweepLaunch &a, const GenEntry *tab, const void *val,
                   const int *idx, void *rbuf, void *zpart, hipStream_t s, LaunchTimer t) {
    constexpr int SL = MP / kGatherCols, S = MP / BigTile<T>::CS;
    constexpr int RS = jgs_split<T, MP>();
    const int steps = (a.L + chunks - 1) / chunks;
    // few (level, slice) workgroups per step leave most CUs idle: split rows.
    // Levels of 512 stream 256 KB per workgroup, too little to pay for the
    // third launch (measured: 6 % faster at one chunk, 19 % slower at 12).
    const bool split = MP >= 1024 && chunks * S < kJgsSplitBelow && zpart;
    SweepLaunch b = a;
    for (int step = 0; step < steps; ++step) {
        // the sweep's launches are timed as one span
        const LaunchTimer t0{step == 0 ? t.start : nullptr, nullptr};
        const LaunchTimer t1{nullptr, step == steps - 1 ? t.stop : nullptr};
        b.fold = step == 0 ? a.fold : 0;
        launch_timed(k_gather_big_jgs<T, MP, NT>, chunks * SL, s, t0, b, chunks, step, tab,
                     (const T *)val, idx, (T *)rbuf);
        if (split) {
            SweepLaunch c = b;
            c.fold = 0;
            launch_timed(k_apply_big<T, MP, false, NT, true, RS>, chunks * S * RS, s,
                         LaunchTimer(), c, (const T *)rbuf, chunks, step, (T *)zpart);
            launch_timed(k_combine_big_jgs<T, MP, RS>, chunks * S + (b.fold ? 1 : 0), s, t1, b,
                         chunks, step, (const T *)zpart);
        } else {
            launch_timed(k_apply_big<T, MP, false, NT, true, 1>, chunks * S + (b.fold ? 1 : 0), s,
                         t1, b, (const T *)rbuf, chunks, step, (T *)nullptr);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T, bool NT>
hipError_t jgs_big_t(int MP, int chunks, const SweepLaunch &a, const GenEntry *tab,
                     const void *val, const int *idx, void *rbuf, void *zpart, hipStream_t s,
                     LaunchTimer t) {
    switch (MP) {
        case 512: return jgs_big<T, 512, NT>(chunks, a, tab, val, idx, rbuf, zpart, s, t);
        case 1024: return jgs_big<T, 1024, NT>(chunks, a, tab, val, idx, rbuf, zpart, s, t);
        case 2048: return jgs_big<T, 2048, NT>(chunks, a, tab, val, idx, rbuf, zpart, s, t);
    }
    return hipErrorInvalidValue;
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
               ? diff_big_t<double>(MP, w, w_prev, parity_a, gA, gB, 2, st, k, part, stream)
               : diff_big_t<float>(MP, w, w_prev, parity_a, gA, gB, 2, st, k, part, stream);
}

hipError_t launch_sweep_jgs_big(int precision_bytes, int MP, bool nt, int chunks,
                                const SweepLaunch &a, const GenEntry *tab, const void *val,
                                const int *idx, void *rbuf, void *zpart, hipStream_t stream,
                                LaunchTimer t) {
    if (!rbuf || chunks < 1 || chunks > a.L) return hipErrorInvalidValue;
    if (precision_bytes == 8)
        return nt ? jgs_big_t<double, true>(MP, chunks, a, tab, val, idx, rbuf, zpart, stream, t)
                  : jgs_big_t<double, false>(MP, chunks, a, tab, val, idx, rbuf, zpart, stream,
                                             t);
    return nt ? jgs_big_t<float, true>(MP, chunks, a, tab, val, idx, rbuf, zpart, stream, t)
              : jgs_big_t<float, false>(MP, chunks, a, tab, val, idx, rbuf, zpart, stream, t);
}

size_t jgs_big_split_bytes(int L, int MP) { return (size_t)kJgsSplit * L * MP * sizeof(double); }

hipError_t launch_diff_big_levels(int precision_bytes, int MP, const void *w, const void *w_prev,
                                  int L, const DevState *st, long long k, double *part,
                                  hipStream_t stream) {
    const int n = L * (MP / kSliceCols);
    return precision_bytes == 8
               ? diff_big_t<double>(MP, w, w_prev, 0, n, 0, 1, st, k, part, stream)
               : diff_big_t<float>(MP, w, w_prev, 0, n, 0, 1, st, k, part, stream);
}

hipError_t launch_residual_big_partials(int precision_bytes, int MP, int groups,
                                        const double *diag, const GenEntry *tab, const double *val,
                                        const int *idx, const void *w, const DevState *st,
                                        long long slot, double *part, hipStream_t stream) {
    return precision_bytes == 8
               ? residual_big_t<double>(MP, groups, diag, tab, val, idx, w, st, slot, part, stream)
               : residual_big_t<float>(MP, groups, diag, tab, val, idx, w, st, slot, part, stream);
}


size_t big_invert_scratch_bytes(int MP, int L) {
    return (size_t)L * MP * 8 + (size_t)L * kPanel * kPanel * 8 + (size_t)L * 4;
}

namespace {

template <int MP>
hipError_t invert_big(const double *diag, const int *sizes, double *W, int L, DevState *st,
                      void *scratch, hipStream_t s) {
    constexpr int NT = MP / kPanel;
    double *dorig = (double *)scratch;
    double *dinv = dorig + (size_t)L * MP;
    int *bad = (int *)(dinv + (size_t)L * kPanel * kPanel);
    const size_t n2 = (size_t)L * MP * MP / 2;
    size_t g = (n2 + kWG - 1) / kWG;
    if (g > 8192) g = 8192;
    if (g * kWG < (size_t)L) g = ((size_t)L + kWG - 1) / kWG;
    hipLaunchKernelGGL((k_binv_init<MP>), dim3((unsigned)g), dim3(kWG), 0, s, diag, sizes, W,
                       dorig, bad, L);
    for (int kb = 0; kb < NT; ++kb) {
        hipLaunchKernelGGL((k_binv_panel<MP>), dim3(L), dim3(64 * inv_waves(kPanel)), 0, s, W,
                           dorig, dinv, bad, kb);
        hipLaunchKernelGGL((k_binv_row<MP>), dim3(L * (NT - 1)), dim3(kWG), 0, s, W, dinv, kb);
        hipLaunchKernelGGL((k_binv_trail<MP>), dim3(L * (NT - 1) * (NT - 1)), dim3(kWG), 0, s, W,
                           kb);
        hipLaunchKernelGGL((k_binv_col<MP>), dim3(L * NT), dim3(kWG), 0, s, W, dinv, kb);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_binv_final<MP>), dim3((unsigned)g), dim3(kWG), 0, s, W, sizes, bad, st, L);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_invert_big(int MP, const double *diag, const int *sizes, double *blk, int L,
                             DevState *st, void *scratch, hipStream_t stream) {
    if (!scratch) return hipErrorInvalidValue;
    switch (MP) {
        case 512: return invert_big<512>(diag, sizes, blk, L, st, scratch, stream);
        case 1024: return invert_big<1024>(diag, sizes, blk, L, st, scratch, stream);
        case 2048: return invert_big<2048>(diag, sizes, blk, L, st, scratch, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace stc
