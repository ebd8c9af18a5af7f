#pragma once
// Device code of the block staircase-splitting solver (gfx950): the kernel
// templates, shared by the launcher files (one translation unit per family,
// compiled in parallel).
//
// One sweep of Algorithm 2 (section 2) is two launches:
//   phase A: every diagonal-only level i (independent):
//              r_i = sum_{k != i} A_{i,k} x_k         (old iterate)
//              z_i = W_i r_i,  W_i = (-A_{i,i})^{-1}
//   phase B: every stair level i, from the fresh phase-A neighbours:
//              r_i = sum_{k = i+-1} A_{i,k} z_k + sum_{|k-i| >= 2} A_{i,k} x_k
//              z_i = W_i r_i
// followed by the normalisation z / e^T z and the change ||z - x||_1.  Here
// A = Q^T, so A_{i,k} v = Q_{k,i}^T v; every product is a non-negative block
// times a non-negative vector (no cancellation).
//
// Layout in HBM (per chain):
//   blk [L][2b+1][MP][MP]  level-major, so one level's blocks are contiguous.
//                          Slot d+b, d != 0, holds Q_{i+d,i} row-major (rows =
//                          states of level i+d, columns = states of level i);
//                          slot b holds (-Q_ii)^{-1} row-major.  The product
//                          with a vector is a column gather: y[j] = sum_r
//                          B[r][j] v[r], so lanes run along a row and every
//                          load is a contiguous 16-byte piece of one row.
//   W   [L][MP]            iterates, zero padded.
//
// Normalisation is lazy and lagged.  The sweep producing W_s reads W_{s-1}
// scaled by kappa_s = 1 / e^T W_{s-2}: the sweep map is linear, so
// x^(s) = W_s / e^T W_s is exactly the normalised iterate of Algorithm 2,
// while e^T W_s = g_s e^T W_{s-1} / e^T W_{s-2} stays bounded (g_s -> 1 at
// the fixed point).  Each launch writes fixed-order per-workgroup partial
// sums of its output and of the change ||x^(s-2) - x^(s-3)||_1; the partials
// of sweep s-1 are reduced by one extra workgroup of the phase-B launch of
// sweep s (or by a one-workgroup finalize launch), which records e^T W_{s-1}
// and applies the device stopping test.  Nothing on the path of a sweep waits
// for a reduction, no workgroup waits on another, and no kernel needs a
// device-wide fence.  The change being measured two sweeps late, the iterates
// rotate through four buffers.
#include <math.h>

#include "stc_internal.h"

namespace stc {

constexpr int kWG = 256;

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    typedef double __attribute__((ext_vector_type(2))) type;
};
template <>
struct Vec16<float> {
    typedef float __attribute__((ext_vector_type(4))) type;
};

// Thread geometry of one level ("team"): CT lanes span a block row with
// 16-byte loads, R row groups (RG requested) split the rows, LPW levels share
// a workgroup.
template <typename T, int MP, int RG = 8>
struct Tile {
    static constexpr int VEC = 16 / (int)sizeof(T);
    static constexpr int CT = MP / VEC;
    static constexpr int TS = (CT * RG <= kWG) ? CT * RG : kWG;
    static constexpr int R = TS / CT;
    static constexpr int RPT = MP / R;
    static constexpr int LPW = kWG / TS;
    static constexpr int PF = RPT < 8 ? RPT : 8;   // W_i rows prefetched per thread
};

// Algorithm 1's chunks: chunk q of `chunks` holds the levels
// jgs_first(q) .. jgs_first(q + 1) - 1.
__device__ inline int jgs_first(int q, int L, int chunks) {
    return (int)((long long)q * L / chunks);
}

// Launch variants: see kVariants in stc_internal.h.

template <typename VT, bool NT>
__device__ inline VT stream_load(const VT *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Device-scope (cross-XCD coherent) relaxed loads and stores, for data that
// another block of the same persistent launch wrote or will read.  COH =
// false gives plain accesses (the producer and consumer are separated by a
// kernel boundary).
template <bool COH, typename T>
__device__ inline T cload(const T *p) {
    if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
}
template <bool COH, typename T>
__device__ inline void cstore(T *p, T v) {
    if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

// Sums for the normalisation e^T z and the change.  Each workgroup of a
// sweep sums the at most LPW * MP terms of its own levels with a plain
// fixed-order tree (error below log2(LPW * MP) units of the last place,
// independent of the chain's length).  The fold of the per-group partials,
// whose count grows with the chain, is compensated: every addition is an
// exact TwoSum whose rounding error is carried in a second word, in a
// fixed order, so the total stays deterministic and its error does not
// grow with the number of groups.
__device__ inline void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

// (hi, lo) += (h2, l2)
__device__ inline void dd_add(double &hi, double &lo, double h2, double l2) {
    double s, e;
    two_sum(hi, h2, s, e);
    hi = s;
    lo = (lo + l2) + e;
}

// (hi, lo) += v, for sequential accumulation in a thread
__device__ inline void dd_acc(double &hi, double &lo, double v) {
    double s, e;
    two_sum(hi, v, s, e);
    hi = s;
    lo += e;
}

// Butterfly over the wave: every lane ends with the same pair (TwoSum is
// symmetric in its arguments: same sum, same exact error).
__device__ inline void wave_sum_dd(double &hi, double &lo) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dd_add(hi, lo, __shfl_xor(hi, o, 64), __shfl_xor(lo, o, 64));
}

// Fixed-order compensated workgroup sum of the pairs (hi, lo); every thread
// gets the same value.  sh holds 4 * kWG / 64 doubles.
__device__ inline double block_sum_dd(double hi, double lo, double *sh) {
    wave_sum_dd(hi, lo);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sh[2 * w] = hi;
        sh[2 * w + 1] = lo;
    }
    __syncthreads();
    double th = sh[0], tl = sh[1];
#pragma unroll
    for (int j = 1; j < kWG / 64; ++j) dd_add(th, tl, sh[2 * j], sh[2 * j + 1]);
    return th + tl;
}

// Two compensated workgroup sums with one pair of barriers (the same
// arithmetic as two block_sum_dd calls).
__device__ inline void block_sum2_dd(double &ah, double al, double &bh, double bl, double *sh) {
    wave_sum_dd(ah, al);
    wave_sum_dd(bh, bl);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sh[4 * w] = ah;
        sh[4 * w + 1] = al;
        sh[4 * w + 2] = bh;
        sh[4 * w + 3] = bl;
    }
    __syncthreads();
    double th = sh[0], tl = sh[1], uh = sh[2], ul = sh[3];
#pragma unroll
    for (int j = 1; j < kWG / 64; ++j) {
        dd_add(th, tl, sh[4 * j], sh[4 * j + 1]);
        dd_add(uh, ul, sh[4 * j + 2], sh[4 * j + 3]);
    }
    ah = th + tl;
    bh = uh + ul;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Plain fixed-order workgroup sum (every thread gets the same value), for
// the few hundred terms of one group.
__device__ inline double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < kWG / 64; ++j) t += sh[j];
    return t;
}

// Two plain fixed-order workgroup sums with one pair of barriers (the same
// arithmetic as two block_sum calls).
__device__ inline void block_sum2(double &a, double &b, double *sh) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sh[w] = a;
        sh[kWG / 64 + w] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int j = 0; j < kWG / 64; ++j) {
        ta += sh[j];
        tb += sh[kWG / 64 + j];
    }
    a = ta;
    b = tb;
}

__device__ inline double block_max(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = sh[0];
#pragma unroll
    for (int j = 1; j < kWG / 64; ++j) t = fmax(t, sh[j]);
    return t;
}

// ---------------------------------------------------------------------------
// half-sweep
// ---------------------------------------------------------------------------
// The work of one workgroup in a half-sweep: LPW levels of one chain
// (team t of group q owns level parity + 2 (q LPW + t)), then the group's
// partial sums into slot slot0 + q.  Used by the single-chain launch and by
// the persistent multi-chain launch.
template <typename T>
struct ChainView {
    const T *blk;
    const T *w_old;          // W_{s-1}
    const T *w_d1, *w_d2;    // W_{s-2}, W_{s-3}: the change of sweep s-2
    T *w_new;                // W_s
    double *part_sum, *part_diff;
    const DevState *st;
    int L, parity, slot0;
    long long s;
};

// Fixed-order sums of per-group partials (same value in every workgroup).
template <bool COH = false>
__device__ inline void partial_sums(const double *ps, const double *pd, int n, bool want_d,
                                    double *sh, double &S, double &D) {
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
    // each thread takes slots j, j + kWG, j + 2 kWG, ... in that order; the
    // loads of U of them are issued before their adds, so a long fold waits
    // for one load round trip per U slots instead of one per slot
    constexpr int U = 8;
    int j = threadIdx.x;
    for (; j + (U - 1) * kWG < n; j += U * kWG) {
        double a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = cload<COH>(ps + j + u * kWG);
            b[u] = want_d ? cload<COH>(pd + j + u * kWG) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dd_acc(s1, c1, a[u]);
            if (want_d) dd_acc(s2, c2, b[u]);
        }
    }
    for (; j < n; j += kWG) {
        dd_acc(s1, c1, cload<COH>(ps + j));
        if (want_d) dd_acc(s2, c2, cload<COH>(pd + j));
    }
    block_sum2_dd(s1, c1, s2, c2, sh);
    S = s1;
    D = want_d ? s2 : 0.0;
}

// Record sweep s in the state: 1 / e^T W_s and the change of sweep s - 2
// (measured during sweep s), then the device stopping test.  Thread 0 only;
// nothing after a stop.
template <bool COH = false>
__device__ inline void record_sweep(DevState *st, long long s, double S, double D, double tol) {
    if (cload<COH>(&st->stop_flag)) return;
    cstore<COH>(&st->last_sweep, s);
    if (!(S > 0.0) || !isfinite(S)) {
        cstore<COH>(&st->status, (int)kDevDegenerate);
        cstore<COH>(&st->stop_sweep, s - 1);
        cstore<COH>(&st->stop_flag, 1);
        return;
    }
    cstore<COH>(&st->inv_sigma[s & kRingMask], 1.0 / S);
    if (s >= 3 && s - 2 > cload<COH>(&st->test_after)) {
        cstore<COH>(&st->diff[(s - 2) & kRingMask], D);
        if (tol > 0.0 && D <= tol) {
            cstore<COH>(&st->stop_sweep, s - 2);
            cstore<COH>(&st->stop_flag, 1);
        }
    }
}

// COH: persistent launch (device-scope accesses for data other blocks of the
// launch write).  LOOP: called from a loop over groups or work items.
template <typename T, int MP, int B, bool PHB, int RG, bool NT, bool COH = false,
          bool LOOP = COH>
__device__ inline void sweep_group(const ChainView<T> &a, int q, bool live, double inv_old,
                                   T *red_base, T *rv_base, double *sh) {
    // persistent launch: live is uniform over the block, and a sweep after
    // the stop changes nothing, so it skips the block streams as well
    if constexpr (COH) {
        if (!live) return;
    }
    using TL = Tile<T, MP, RG>;
    using VT = typename Vec16<T>::type;
    constexpr int NB = 2 * B + 1;
    constexpr int VEC = TL::VEC, CT = TL::CT, R = TL::R, RPT = TL::RPT, TS = TL::TS,
                  LPW = TL::LPW, PF = TL::PF;
    constexpr size_t BS = (size_t)MP * MP;

    const DevState *st = a.st;
    int tid = threadIdx.x;
    if constexpr (LOOP) {
        // opaque to the optimiser: in the persistent and work-list loops the
        // per-thread row offsets would otherwise be hoisted and held across
        // every item, raising the registers and cutting the resident blocks
        asm volatile("" : "+v"(tid));
    }
    const int team = tid / TS, tt = tid - team * TS;
    const int c = tt % CT, g = tt / CT;
    T *red = red_base + team * (R * MP);     // [R][MP] of this team
    T *rv = rv_base + team * MP;             // [MP]
    const int i = a.parity + 2 * (q * LPW + team);
    const bool active = i < a.L;
    const int ic = active ? i : a.parity;   // a valid level for idle teams
    const T *w_old = a.w_old;
    T *w_new = a.w_new;
    const T *base = a.blk + (size_t)ic * NB * BS;
    const T sc = (T)inv_old;

    // r_i: gather of the off-diagonal blocks of block row i of A.  The loop
    // has no branches, so all block loads of the level are in flight at once;
    // a neighbour outside [0, L) has an all-zero stored block and weight 0,
    // and reads the old iterate at level ic instead (always written and
    // finite, so 0 * value stays 0; the fresh buffer may still hold stale or
    // uninitialised values there).
    // (persistent launch: the neighbour values are device-scope loads, since
    // another block of the same launch may have written them)
    VT acc = (VT)(T)0;
#pragma unroll
    for (int d = -B; d <= B; ++d) {
        if (d == 0) continue;
        const int k = ic + d;
        const bool in = (k >= 0) && (k < a.L);
        const bool fresh = PHB && (d == 1 || d == -1);
        const T *v = in ? (fresh ? (const T *)w_new : w_old) + (size_t)k * MP
                        : w_old + (size_t)ic * MP;
        const T vs = in ? (fresh ? (T)1 : sc) : (T)0;
        const T *gb = base + (size_t)(d + B) * BS + c * VEC;
#pragma unroll
        for (int qq = 0; qq < RPT; ++qq) {
            const int row = g + R * qq;
            const VT blkv = stream_load<VT, NT>((const VT *)(gb + (size_t)row * MP));
            acc += blkv * (cload<COH>(v + row) * vs);
        }
    }
    // rows of W_i fetched before the reduction, so they stream meanwhile
    VT vpre[PF];
    const T *wb = base + (size_t)B * BS + c * VEC;
#pragma unroll
    for (int qq = 0; qq < PF; ++qq)
        vpre[qq] = stream_load<VT, NT>((const VT *)(wb + (size_t)(g + R * qq) * MP));

#pragma unroll
    for (int e = 0; e < VEC; ++e) red[g * MP + c * VEC + e] = acc[e];
    __syncthreads();
    // a team may be narrower than a block row (small blocks): stride by TS
#pragma unroll
    for (int e = tt; e < MP; e += TS) {
        T r = 0;
#pragma unroll
        for (int gg = 0; gg < R; ++gg) r += red[gg * MP + e];
        rv[e] = r;
    }
    __syncthreads();

    // z_i = W_i r_i
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
    __syncthreads();

    double zs = 0.0, dd = 0.0;
    if (live && active) {
#pragma unroll
        for (int e = tt; e < MP; e += TS) {
            T z = 0;
#pragma unroll
            for (int gg = 0; gg < R; ++gg) z += red[gg * MP + e];
            cstore<COH>(w_new + (size_t)i * MP + e, z);
            zs += (double)z;
            if (a.s >= 3) {
                // ||x^(s-2) - x^(s-3)||_1 terms: both scales are recorded by now
                const double i2 = cload<COH>(&st->inv_sigma[(a.s - 2) & kRingMask]);
                const double i3 = cload<COH>(&st->inv_sigma[(a.s - 3) & kRingMask]);
                dd += fabs((double)cload<COH>(a.w_d1 + (size_t)i * MP + e) * i2 -
                           (double)cload<COH>(a.w_d2 + (size_t)i * MP + e) * i3);
            }
        }
    }
    double S = zs, D = dd;
    block_sum2(S, D, sh);
    if (live && tid == 0) {
        cstore<COH>(a.part_sum + a.slot0 + q, S);
        cstore<COH>(a.part_diff + a.slot0 + q, D);
    }
    __syncthreads();   // the LDS may be reused by the next group
}

// The extra workgroup of a phase-B launch: reduce sweep s-1's partials and
// record them (it runs beside the streaming workgroups, off their path).
__device__ inline void fold_previous(const SweepLaunch &a, double *sh) {
    double S, D;
    partial_sums(a.prev_sum, a.prev_diff, a.prev_nslots, true, sh, S, D);
    if (threadIdx.x == 0) record_sweep(a.st, a.s - 1, S, D, a.tol);
}

template <typename T>
__device__ inline ChainView<T> view_of(const SweepLaunch &a) {
    ChainView<T> v;
    v.blk = (const T *)a.blk;
    v.w_old = (const T *)a.w_old;
    v.w_d1 = (const T *)a.w_d1;
    v.w_d2 = (const T *)a.w_d2;
    v.w_new = (T *)a.w_new;
    v.part_sum = a.part_sum;
    v.part_diff = a.part_diff;
    v.st = a.st;
    v.L = a.L;
    v.parity = a.parity;
    v.slot0 = a.slot0;
    v.s = a.s;
    return v;
}

template <typename T, int MP, int B, bool PHB, int RG, bool NT>
__global__ __launch_bounds__(kWG) void k_sweep(SweepLaunch a) {
    using TL = Tile<T, MP, RG>;
    __shared__ T red[TL::LPW * TL::R * MP];
    __shared__ T rv[TL::LPW * MP];
    __shared__ double sh[4 * kWG / 64];
    int q = blockIdx.x;
    if (PHB && a.fold) {
        // the reduction workgroup is dispatched first, so it runs beside the
        // whole phase instead of after its last wave of groups
        if (q == 0) {
            fold_previous(a, sh);
            return;
        }
        --q;
    }
    // a sweep queued after the device stopping test fired changes nothing
    const bool live = a.st->stop_flag == 0;
    const double kappa = a.st->inv_sigma[(a.s - 2) & kRingMask];
    sweep_group<T, MP, B, PHB, RG, NT>(view_of<T>(a), q, live, kappa, red, rv, sh);
}

// ---------------------------------------------------------------------------
// a burst of sweeps in one persistent cooperative launch
// ---------------------------------------------------------------------------
// The dependencies of a sweep are local: a level of phase A reads the levels
// next to it from the previous sweep, a level of phase B the fresh phase-A
// levels next to it.  Block g owns a contiguous range of the groups of each
// phase and publishes "phase A (or B) of sweep j done" in its flags; before
// the groups that read levels of another block it waits for that block's
// flag, and it runs the groups that only read its own levels first.  An
// extra block, the folder, reduces a sweep's partials once every block has
// published it and records the sweep; the scale 1 / e^T W_{s-2} that sweep s
// needs is therefore recorded a full sweep before it is read.  Every wait is bounded by wall
// clock time: past it the launch is marked aborted (status kDevTimeout) and
// every block returns.  Data that crosses blocks is read and written with
// device-scope relaxed accesses (coherent across the XCDs' L2 caches), and a
// block's stores are complete before its flag is set.

// Upper bound on the polls of one wait (each poll sleeps about 128 clocks,
// so this is several seconds: past the wall clock bound).
constexpr long long kFlowMaxSpins = 1ll << 26;

// Thread 0 waits until *p >= target; false if the launch aborted.
__device__ inline bool flow_wait(const unsigned *p, unsigned target, const FlowLaunch &f,
                                 int *sh_ok) {
    if (threadIdx.x == 0) {
        int ok = 1;
        if (cload<true>(p) < target) {
            unsigned *abort_flag = f.flags + 2 * f.G + 1;
            const long long t0 = (long long)wall_clock64();
            long long spins = 0;
            while (cload<true>(p) < target) {
                if (cload<true>(abort_flag)) {
                    ok = 0;
                    break;
                }
                // wall clock bound, and a count bound in case the clock stalls
                if ((long long)wall_clock64() - t0 > f.timeout_ticks || ++spins > kFlowMaxSpins) {
                    cstore<true>(&f.st->status, (int)kDevTimeout);
                    cstore<true>(&f.st->stop_flag, 1);
                    cstore<true>(abort_flag, 1u);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        *sh_ok = ok;
    }
    __syncthreads();
    const bool ok = *sh_ok != 0;
    __syncthreads();
    return ok;
}

// Every wave's stores are complete, then thread 0 sets the flag.
__device__ inline void flow_publish(unsigned *flag, unsigned v) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) cstore<true>(flag, v);
}

// Block of group q of a phase with n groups split over G blocks
// (block g owns groups [g n / G, (g + 1) n / G)).
__device__ inline int flow_owner(int q, int n, int G) {
    return (int)(((long long)(q + 1) * G - 1) / n);
}

// The folder (block G): record each sweep once every block has finished it.
// It polls the blocks' flags; no atomics (one counter hit by every block of
// every sweep serialises at the memory side).
__device__ inline void flow_fold(const FlowLaunch &f, double *sh, int *sh_ok) {
    const unsigned *fb = f.flags + f.G;
    unsigned *folded = f.flags + 2 * f.G;
    const unsigned *abort_flag = f.flags + 2 * f.G + 1;
    const int nslots = f.groups_a + f.groups_b;
    for (int j = 1; j <= f.n; ++j) {
        const long long s = f.s0 + j;
        long long t0 = 0;
        for (long long spin = 0;; ++spin) {
            int mine = 1;
            for (int g = threadIdx.x; g < f.G; g += kWG)
                if (cload<true>(fb + g) < (unsigned)j) {
                    mine = 0;
                    break;
                }
            if (__syncthreads_and(mine)) break;
            if (threadIdx.x == 0) {
                int ok = 1;
                if (spin == 0) t0 = (long long)wall_clock64();
                if (cload<true>(abort_flag)) {
                    ok = 0;
                } else if ((long long)wall_clock64() - t0 > f.timeout_ticks ||
                           spin > kFlowMaxSpins) {
                    cstore<true>(&f.st->status, (int)kDevTimeout);
                    cstore<true>(&f.st->stop_flag, 1);
                    cstore<true>(f.flags + 2 * f.G + 1, 1u);
                    ok = 0;
                }
                *sh_ok = ok;
                __builtin_amdgcn_s_sleep(2);
            }
            __syncthreads();
            const bool ok = *sh_ok != 0;
            __syncthreads();
            if (!ok) return;
        }
        double S, D;
        partial_sums<true>(f.part_sum + (s & 1) * f.nparts, f.part_diff + (s & 1) * f.nparts,
                           nslots, true, sh, S, D);
        if (threadIdx.x == 0) {
            record_sweep<true>(f.st, s, S, D, f.tol);
            __builtin_amdgcn_s_waitcnt(0);
            cstore<true>(folded, (unsigned)j);
        }
        __syncthreads();
    }
}

template <typename T>
__device__ inline ChainView<T> flow_view(const FlowLaunch &f, long long s, int parity,
                                         int slot0) {
    ChainView<T> v;
    v.blk = (const T *)f.blk;
    v.w_old = (const T *)f.w[(s - 1) & 3];
    v.w_d1 = (const T *)f.w[(s - 2) & 3];
    v.w_d2 = (const T *)f.w[(s - 3) & 3];
    v.w_new = (T *)f.w[s & 3];
    v.part_sum = f.part_sum + (s & 1) * f.nparts;
    v.part_diff = f.part_diff + (s & 1) * f.nparts;
    v.st = f.st;
    v.L = f.L;
    v.parity = parity;
    v.slot0 = slot0;
    v.s = s;
    return v;
}

// One phase of sweep j for block g: the groups whose neighbour levels are all
// this block's first, then (after waiting for the other blocks' flags at
// `need`) the rest.  PHB: the neighbours of a level are phase-A levels of
// this sweep (flag fa >= j); else phase-B levels of the previous sweep
// (flag fb >= j - 1, which also covers that block's phase A).
template <typename T, int MP, int B, bool PHB, int RG, bool NT>
__device__ inline bool flow_phase(const FlowLaunch &f, const ChainView<T> &v, int g, int j,
                                  bool live, double kappa, T *red, T *rv, double *sh,
                                  int *sh_ok) {
    constexpr int LPW = Tile<T, MP, RG>::LPW;
    const int G = f.G;
    const int par = v.parity, opar = 1 - par;
    const int n = PHB ? f.groups_b : f.groups_a;
    const int on = PHB ? f.groups_a : f.groups_b;   // groups of the other phase
    const int lo = (int)((long long)g * n / G), hi = (int)((long long)(g + 1) * n / G);
    const unsigned *flag = PHB ? f.flags : f.flags + G;
    const unsigned target = PHB ? (unsigned)j : (unsigned)(j - 1);
    // owners of the levels within B of group q's levels, other than g
    auto owner_of_level = [&](int l, int p, int np) {
        return flow_owner(((l - p) >> 1) / LPW, np, G);
    };
    auto external = [&](int q, int *wl, int *wr) {
        const int first = par + 2 * q * LPW;
        const int last = min(par + 2 * (q * LPW + LPW - 1), (f.L - 1 - par) / 2 * 2 + par);
        int l = g, r = g;
        for (int d = 1; d <= B; ++d) {
            const int pl = first - d, pr = last + d;
            const int pp = (d & 1) ? opar : par;
            const int np = (d & 1) ? on : n;
            if (pl >= 0) l = min(l, owner_of_level(pl, pp, np));
            if (pr < f.L) r = max(r, owner_of_level(pr, pp, np));
        }
        *wl = l;
        *wr = r;
        return l != g || r != g;
    };
    // interior groups first (lo+1 .. hi-2), then the two end groups (the
    // order only matters for overlap: the end groups are the ones that
    // usually read another block's levels); before the first group that
    // does, wait for every block that any group of the range reads from
    const int cnt = hi - lo;
    bool waited = target == 0;
    for (int k = 0; k < cnt; ++k) {
        const int q = cnt <= 2 ? lo + k : (k < cnt - 2 ? lo + 1 + k : (k == cnt - 2 ? lo : hi - 1));
        int wl, wr;
        if (!waited && external(q, &wl, &wr)) {
            int wmin = g, wmax = g;
            for (int qq = lo; qq < hi; ++qq) {
                int l2, r2;
                external(qq, &l2, &r2);
                wmin = min(wmin, l2);
                wmax = max(wmax, r2);
            }
            for (int w = wmin; w <= wmax; ++w)
                if (w != g && !flow_wait(flag + w, target, f, sh_ok)) return false;
            waited = true;
        }
        sweep_group<T, MP, B, PHB, RG, NT, true>(v, q, live, kappa, red, rv, sh);
    }
    return true;
}

template <typename T, int MP, int B, int RG, bool NT>
__global__ __launch_bounds__(kWG) void k_sweep_flow(FlowLaunch f) {
    using TL = Tile<T, MP, RG>;
    __shared__ T red[TL::LPW * TL::R * MP];
    __shared__ T rv[TL::LPW * MP];
    __shared__ double sh[4 * kWG / 64];
    __shared__ int sh_ok, sh_live;
    __shared__ double sh_kappa;
    if ((int)blockIdx.x == f.G) {
        flow_fold(f, sh, &sh_ok);
        return;
    }
    // logical block: blocks are handed to the 8 XCDs in turn, so number
    // them XCD by XCD and neighbouring ranges mostly share an XCD's L2
    const int b = blockIdx.x, G = f.G, per = G / 8, rem = G % 8, x = b % 8;
    const int g = x * per + min(x, rem) + b / 8;
    unsigned *fa = f.flags, *fb = f.flags + f.G;
    const unsigned *folded = f.flags + 2 * f.G;
    const int pA = f.parity_a, pB = 1 - pA;
    for (int j = 1; j <= f.n; ++j) {
        const long long s = f.s0 + j;
        // the scale of sweep s (1 / e^T W_{s-2}) is recorded by the folder
        if (j >= 3 && !flow_wait(folded, (unsigned)(j - 2), f, &sh_ok)) return;
        if (threadIdx.x == 0) {
            sh_live = cload<true>(&f.st->stop_flag) == 0;
            sh_kappa = cload<true>(&f.st->inv_sigma[(s - 2) & kRingMask]);
        }
        __syncthreads();
        const bool live = sh_live != 0;
        const double kappa = sh_kappa;
        __syncthreads();
        if (!flow_phase<T, MP, B, false, RG, NT>(f, flow_view<T>(f, s, pA, 0), g, j, live, kappa,
                                                 red, rv, sh, &sh_ok))
            return;
        flow_publish(fa + g, (unsigned)j);
        if (!flow_phase<T, MP, B, true, RG, NT>(f, flow_view<T>(f, s, pB, f.groups_a), g, j, live,
                                                kappa, red, rv, sh, &sh_ok))
            return;
        flow_publish(fb + g, (unsigned)j);
    }
}

// ---------------------------------------------------------------------------
// half-sweep with sparse off-diagonal blocks (column-major ELL per block):
// the nonzeros of block Q_{i+d,i} are grouped by output column j, padded to
// 4 Kq slots with Kq = ceil(longest column / 4), and stored by slot quads:
// slot 4 kq + t of column j at [kq][j][t], a value and the 8-bit row index r
// of the source vector v_{i+d}.  A lane owns a column and reads a quad with
// one 16-byte (FP32) or two 16-byte (FP64) value loads and one 4-byte index
// load; consecutive lanes read consecutive quads, so loads are coalesced.
// The source vectors are staged in LDS for the row gather; W_i stays dense.
// The summation order is fixed (deterministic).
// ---------------------------------------------------------------------------
template <typename T, int MP, int B, bool PHB>
__device__ inline void sweep_group_ell(const ChainView<T> &a, const EllEntry *tab,
                                       const T *ell_val, const unsigned char *ell_idx, int q,
                                       bool live, double inv_old, T *red_base, T *rv_base,
                                       T *src_base, unsigned short *base_base, double *sh) {
    using TL = Tile<T, MP, 8>;
    using VT = typename Vec16<T>::type;
    constexpr int NB = 2 * B + 1;
    constexpr int VEC = TL::VEC, CT = TL::CT, R = TL::R, RPT = TL::RPT, TS = TL::TS,
                  LPW = TL::LPW, PF = TL::PF;
    constexpr int G = TS / MP;            // groups splitting the ELL slots of a column
    constexpr size_t BS = (size_t)MP * MP;
    static_assert(G >= 1, "team narrower than a block");

    const DevState *st = a.st;
    const int tid = threadIdx.x;
    const int team = tid / TS, tt = tid - team * TS;
    const int c = tt % CT, g = tt / CT;
    T *red = red_base + team * (R * MP);
    T *rv = rv_base + team * MP;
    T *src = src_base + team * (2 * B * MP);   // [2B][MP] scaled source vectors
    constexpr int NBASE = MP / 4 + 1;          // round offsets per block, at most
    unsigned short *base = base_base + team * (2 * B * NBASE);
    const int i = a.parity + 2 * (q * LPW + team);
    const bool active = i < a.L;
    const int ic = active ? i : a.parity;
    const T *w_old = a.w_old;
    T *w_new = a.w_new;
    const T sc = (T)inv_old;
    const T *wb = a.blk + ((size_t)ic * NB + B) * BS + c * VEC;

    // the table entries of the level's off-diagonal blocks, and this lane's
    // column quad counts (blocks of 128, upper half: also those of column
    // j - 64, whose ballot counts the lower half's quads of a round)
    const int j = tt % MP, gg0 = tt / MP;
    EllEntry te[2 * B];
    int qj[2 * B], qlow[2 * B];
#pragma unroll
    for (int slot = 0; slot < 2 * B; ++slot) {
        const int d = slot < B ? slot - B : slot - B + 1;
        te[slot] = tab[(size_t)ic * NB + (d + B)];
        const unsigned char *qc = ell_idx + te[slot].meta;
        const bool present = te[slot].Kq > 0;
        qj[slot] = present ? qc[j] : 0;
        qlow[slot] = (MP > 64 && present && j >= 64) ? qc[j - 64] : 0;
    }
    // rows of W_i stream while the sparse part runs
    VT vpre[PF];
#pragma unroll
    for (int qq = 0; qq < PF; ++qq)
        vpre[qq] = stream_load<VT, true>((const VT *)(wb + (size_t)(g + R * qq) * MP));

    // stage the source vectors (scaled; zero outside [0, L)) and the blocks'
    // round offsets base_t
    for (int e = tt; e < 2 * B * MP; e += TS) {
        const int slot = e / MP, r = e - slot * MP;
        const int d = slot < B ? slot - B : slot - B + 1;   // -B..-1, 1..B
        const int k = ic + d;
        T v = 0;
        if (k >= 0 && k < a.L) {
            const bool fresh = PHB && (d == 1 || d == -1);
            v = fresh ? w_new[(size_t)k * MP + r] : w_old[(size_t)k * MP + r] * sc;
        }
        src[e] = v;
    }
    for (int e = tt; e < 2 * B * NBASE; e += TS) {
        const int slot = e / NBASE, t = e - slot * NBASE;
        const EllEntry te2 = tab[(size_t)ic * NB + (slot < B ? slot : slot + 1)];
        if (te2.Kq > 0 && t <= te2.Kq)
            base[e] = ((const unsigned short *)(ell_idx + te2.meta + MP))[t];
    }
    __syncthreads();

    // r_i[j] = sum_d sum_k val[k][j] * v_{i+d}[idx[k][j]], a quad of slots per load.
    // Round t of a block holds quad t of the columns that still have one; a
    // lane finds its quad's place from ballots of the lanes of its segment
    // (the MP lanes, at most one wave, that share its rounds).  Each pass
    // keeps U quads of one block in flight (the gather is otherwise bound by
    // one load round trip per quad); the sums keep the quad order, so the
    // result does not depend on U.
    constexpr int SEG = MP < 64 ? MP : 64;
    const int lane = threadIdx.x & 63;
    const unsigned long long seg =
        SEG == 64 ? ~0ull : (((1ull << (SEG & 63)) - 1ull) << (lane & ~(SEG - 1)));
    const unsigned long long below = (1ull << lane) - 1ull;
    T accs = 0;
#pragma unroll
    for (int slot = 0; slot < 2 * B; ++slot) {
        const EllEntry e = te[slot];
        const T *sv = src + slot * MP;
        const unsigned short *bt = base + slot * NBASE;
        constexpr int U = sizeof(T) == 8 ? 2 : 4;   // FP64 quads hold twice the registers
        // the loop bound is uniform over a segment, so each ballot sees all of it
        for (int kq0 = gg0; kq0 < e.Kq; kq0 += G * U) {
            unsigned int r4[U];
            T v[U][4];
            bool on[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kq = kq0 + u * G;
                on[u] = kq < qj[slot];
                int rank = __popcll(__ballot(on[u]) & seg & below);
                if constexpr (MP > 64) rank += __popcll(__ballot(kq < qlow[slot]) & seg);
                if (on[u]) {
                    const size_t o = (size_t)e.off + ((size_t)bt[kq] + rank) * 4;
                    r4[u] = __builtin_nontemporal_load((const unsigned int *)(ell_idx + o));
                    if constexpr (sizeof(T) == 8) {
                        const VT v01 = __builtin_nontemporal_load((const VT *)(ell_val + o));
                        const VT v23 = __builtin_nontemporal_load((const VT *)(ell_val + o + 2));
                        v[u][0] = v01[0], v[u][1] = v01[1], v[u][2] = v23[0], v[u][3] = v23[1];
                    } else {
                        const VT v4 = __builtin_nontemporal_load((const VT *)(ell_val + o));
                        v[u][0] = v4[0], v[u][1] = v4[1], v[u][2] = v4[2], v[u][3] = v4[3];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (on[u])
                    accs += v[u][0] * sv[r4[u] & 0xff] + v[u][1] * sv[(r4[u] >> 8) & 0xff] +
                            v[u][2] * sv[(r4[u] >> 16) & 0xff] + v[u][3] * sv[r4[u] >> 24];
        }
    }
    red[gg0 * MP + j] = accs;
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
        const VT wv = (qq < PF) ? vpre[qq < PF ? qq : 0]
                                : stream_load<VT, true>((const VT *)(wb + (size_t)row * MP));
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
    const double S = block_sum(zs, sh);
    const double D = block_sum(dd, sh);
    if (live && tid == 0) {
        a.part_sum[a.slot0 + q] = S;
        a.part_diff[a.slot0 + q] = D;
    }
}

template <typename T, int MP, int B, bool PHB>
__global__ __launch_bounds__(kWG) void k_sweep_ell(SweepLaunch a, const EllEntry *tab,
                                                    const void *ell_val,
                                                    const unsigned char *ell_idx) {
    using TL = Tile<T, MP, 8>;
    __shared__ T red[TL::LPW * TL::R * MP];
    __shared__ T rv[TL::LPW * MP];
    __shared__ T src[TL::LPW * 2 * B * MP];
    __shared__ unsigned short base[TL::LPW * 2 * B * (MP / 4 + 1)];
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
    sweep_group_ell<T, MP, B, PHB>(view_of<T>(a), tab, (const T *)ell_val, ell_idx, q, live,
                                   kappa, red, rv, src, base, sh);
}

// ---------------------------------------------------------------------------
// many chains: one persistent launch per half-sweep over a work list of
// (chain, group) items; each chain's sweep number comes from its own state
// ---------------------------------------------------------------------------
// One launch per block size present (a kernel per block size keeps each one
// at its own register count; one kernel for all sizes took the largest).
// cls: {offset, count} of this block size's items in the work list (read
// on the device, so a captured graph stays valid when the lists change).
// j: the sweep's index in its burst; each chain produces sweep
// s = burst_base + j (burst_base is fixed for the burst, so every workgroup
// agrees on s while the reduction items below update the chain's state).
// Phase A's first items (group < 0) reduce each chain's sweep s - 1 and
// record it, beside the streaming items: sweep s reads the scale of sweep
// s - 2 only, so the record of s - 1 is needed only from sweep s + 1 on.  A
// stop recorded there (sweep s - 3 met the test) may leave sweep s partly
// written; its buffer is not the stop sweep's, and sweep s + 1, which would
// overwrite that, sees the stop flag at its start.
template <typename T, int MP, int B, bool PHB, int RG, bool NT>
__global__ __launch_bounds__(kWG) void k_batch_sweep(const ChainDesc *chains,
                                                      const WorkItem *items, const int *cls,
                                                      int j) {
    using TL = Tile<T, MP, RG>;
    __shared__ T red[TL::LPW * TL::R * MP];
    __shared__ T rv[TL::LPW * MP];
    __shared__ double sh[4 * kWG / 64];
    const int off = cls[0], n = cls[1];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const WorkItem w = items[off + it];
        const ChainDesc &d = chains[w.chain];
        DevState *st = d.st;
        const long long s = st->burst_base + j;
        if (w.group < 0) {
            if (!PHB && j > 0) {
                double S, D;
                const size_t prev = (size_t)((s - 1) & 1) * d.nparts;
                partial_sums(d.part_sum + prev, d.part_diff + prev, d.groups_a + d.groups_b, true,
                             sh, S, D);
                if (threadIdx.x == 0) record_sweep(st, s - 1, S, D, d.tol);
                __syncthreads();   // sh is reused by the next item
            }
            continue;
        }
        const bool live = st->stop_flag == 0;
        ChainView<T> v;
        v.blk = (const T *)d.blk;
        v.w_old = (const T *)d.w[(s + 3) & 3];   // W_{s-1}
        v.w_d1 = (const T *)d.w[(s + 2) & 3];    // W_{s-2}
        v.w_d2 = (const T *)d.w[(s + 1) & 3];    // W_{s-3}
        v.w_new = (T *)d.w[s & 3];
        v.part_sum = d.part_sum + (size_t)(s & 1) * d.nparts;
        v.part_diff = d.part_diff + (size_t)(s & 1) * d.nparts;
        v.st = st;
        v.L = d.L;
        v.parity = PHB ? 1 - d.parity_a : d.parity_a;
        v.slot0 = PHB ? d.groups_a : 0;
        v.s = s;
        const double inv_old = st->inv_sigma[(s - 2) & kRingMask];   // kappa_s
        for (int q = w.group; q < w.group + w.count; ++q)
            sweep_group<T, MP, B, PHB, RG, NT, false, true>(v, q, live, inv_old, red, rv, sh);
    }
}

// e^T W_s and the change of sweep s-1 from the partials of both phases
// (fixed order), then the device stopping test.  One workgroup per chain.
__device__ inline void finalize_chain(const double *part_sum, const double *part_diff,
                                      int nslots, DevState *st, long long s, double tol,
                                      double *sh) {
    double S, D;
    partial_sums(part_sum, part_diff, nslots, true, sh, S, D);
    if (threadIdx.x == 0) record_sweep(st, s, S, D, tol);
}

// One workgroup: fixed-order sum (and max) of per-group partials for the
// residual, change and load kernels.
enum ReduceMode { kReduceResidual = 0, kReduceDiff = 1, kReduceLoad = 2 };

// ---------------------------------------------------------------------------
// residual ||Q^T x||_1 in FP64: (Q^T x)_i = sum_{d != 0} Q_{i+d,i}^T x_{i+d} + Q_ii^T x_i
// ---------------------------------------------------------------------------
template <typename T, int MP, int B>
__global__ __launch_bounds__(kWG) void k_residual(const double *blk, const double *diag,
                                                   const T *w, int L, const DevState *st,
                                                   long long slot, double *part) {
    using TL = Tile<double, MP, 8>;
    using VT = typename Vec16<double>::type;
    constexpr int NB = 2 * B + 1;
    constexpr int VEC = TL::VEC, CT = TL::CT, R = TL::R, RPT = TL::RPT, TS = TL::TS,
                  LPW = TL::LPW;
    constexpr size_t BS = (size_t)MP * MP;
    __shared__ double red[LPW][R][MP];
    __shared__ double sh[4 * kWG / 64];

    const int tid = threadIdx.x;
    const int team = tid / TS, tt = tid - team * TS;
    const int c = tt % CT, g = tt / CT;
    const int i = blockIdx.x * LPW + team;
    const bool active = i < L;
    const double inv = slot < 0 ? 1.0 : st->inv_sigma[slot & kRingMask];

    VT acc = (VT)0.0;
    if (active) {
#pragma unroll
        for (int d = -B; d <= B; ++d) {
            const int k = i + d;
            if (k < 0 || k >= L) continue;
            const T *v = w + (size_t)k * MP;
            const double *gb = (d == 0 ? diag + (size_t)i * BS
                                       : blk + ((size_t)i * NB + (d + B)) * BS) + c * VEC;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int row = g + R * q;
                const VT bv = stream_load<VT, true>((const VT *)(gb + (size_t)row * MP));
                acc += bv * ((double)v[row] * inv);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) red[team][g][c * VEC + e] = acc[e];
    __syncthreads();
    double r = 0.0;
    if (active && tt < MP) {
        double t = 0.0;
#pragma unroll
        for (int gg = 0; gg < R; ++gg) t += red[team][gg][tt];
        r = fabs(t);
    }
    const double S = block_sum(r, sh);
    if (tid == 0) part[blockIdx.x] = S;
}

// ---------------------------------------------------------------------------
// change ||x^(k) - x^(k-1)||_1 of one sweep, per workgroup of the sweep
// kernels' geometry (same levels per group, same slots, same fixed-order
// sums), so it is bitwise the value the partials of sweep k+2 carry.  Used
// at the end of a burst for the last two sweeps.
// ---------------------------------------------------------------------------
template <typename T, int MP, int RG>
__global__ __launch_bounds__(kWG) void k_diff(const T *w, const T *wp, const DevState *st,
                                               long long k, int L, int parity_a, int groups_a,
                                               double *part) {
    using TL = Tile<T, MP, RG>;
    __shared__ double sh[4 * kWG / 64];
    const int tid = threadIdx.x;
    const int team = tid / TL::TS, tt = tid - team * TL::TS;
    const bool in_a = (int)blockIdx.x < groups_a;
    const int q = in_a ? blockIdx.x : blockIdx.x - groups_a;
    const int parity = in_a ? parity_a : 1 - parity_a;
    const int i = parity + 2 * (q * TL::LPW + team);
    // the same terms, order and sums as the sweep kernels' change
    double dd = 0.0;
    if (i < L) {
        const double i2 = st->inv_sigma[k & kRingMask];
        const double i3 = st->inv_sigma[(k - 1) & kRingMask];
#pragma unroll
        for (int e = tt; e < MP; e += TL::TS)
            dd += fabs((double)w[(size_t)i * MP + e] * i2 - (double)wp[(size_t)i * MP + e] * i3);
    }
    const double D = block_sum(dd, sh);
    if (tid == 0) part[blockIdx.x] = D;
}

// ---------------------------------------------------------------------------
// compact FP64 vector -> padded iterate W (type T); partial sums and a flag
// for negative or non-finite entries (k_reduce then records 1/e^T W)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kWG) void k_load(const double *x, const long long *off,
                                               const int *sizes, int L, int MP, T *w,
                                               double *part, int slot) {
    __shared__ double sh[4 * kWG / 64];
    const size_t n = (size_t)L * MP;
    double s = 0.0, sc = 0.0, bad = 0.0;
    for (size_t j = blockIdx.x * (size_t)kWG + threadIdx.x; j < n; j += (size_t)gridDim.x * kWG) {
        const int lev = (int)(j / MP), col = (int)(j - (size_t)lev * MP);
        double v = 0.0;
        if (col < sizes[lev]) v = x[off[lev] + col];
        if (!isfinite(v) || (slot >= 0 && !(v >= 0.0))) {
            bad = 1.0;
            v = 0.0;
        }
        const T t = (T)v;
        w[j] = t;
        dd_acc(s, sc, (double)t);
    }
    s = block_sum_dd(s, sc, sh);
    bad = block_max(bad, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s;
        part[2 * blockIdx.x + 1] = bad;
    }
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_store(const T *w, const long long *off, const int *sizes,
                                                int L, int MP, const DevState *st, long long slot,
                                                double *x) {
    const double inv = st->inv_sigma[slot & kRingMask];
    const size_t n = (size_t)L * MP;
    for (size_t j = blockIdx.x * (size_t)kWG + threadIdx.x; j < n; j += (size_t)gridDim.x * kWG) {
        const int lev = (int)(j / MP), col = (int)(j - (size_t)lev * MP);
        if (col < sizes[lev]) x[off[lev] + col] = (double)w[j] * inv;
    }
}

// ---------------------------------------------------------------------------
// W_i = (-Q_ii)^{-1} by Gauss-Jordan elimination in LDS, one level per group.
// -Q_ii is a diagonally dominant M-matrix (its rows sum to the rate leaving
// the level), so no pivoting is needed and every pivot is positive; a pivot
// that is not clearly positive marks the block singular.  Padding rows and
// columns are carried as an identity and written back as zeros.
// ---------------------------------------------------------------------------
template <int MP>
__global__ __launch_bounds__(kWG) void k_invert(const double *diag, const int *sizes,
                                                 double *blk, int NB, int B, DevState *st) {
    constexpr int LD = MP + 1;
    __shared__ double a[MP * LD];
    __shared__ double colk[MP];
    __shared__ double rowk[MP];
    __shared__ int bad;
    const int i = blockIdx.x;
    const int n = sizes[i];
    const double *Q = diag + (size_t)i * MP * MP;
    if (threadIdx.x == 0) bad = 0;
    for (int idx = threadIdx.x; idx < MP * MP; idx += kWG) {
        const int r = idx / MP, c = idx - r * MP;
        double v;
        if (r < n && c < n) v = -Q[idx];
        else v = (r == c) ? 1.0 : 0.0;
        a[r * LD + c] = v;
    }
    __syncthreads();
    for (int k = 0; k < MP; ++k) {
        const double p = a[k * LD + k];
        if (threadIdx.x < MP) {
            colk[threadIdx.x] = a[threadIdx.x * LD + k];
            rowk[threadIdx.x] = a[k * LD + threadIdx.x];
        }
        if (threadIdx.x == 0) {
            // relative to the row's total rate, which equals the original diagonal
            // up to the eliminated part; a non-positive or vanishing pivot means the
            // level has a closed set of states
            double scale = 0.0;
            for (int c = k; c < MP; ++c) scale += fabs(a[k * LD + c]);
            if (!(p > 1e-13 * scale) || !isfinite(p)) bad = 1;
        }
        __syncthreads();
        const double pinv = 1.0 / p;
        for (int idx = threadIdx.x; idx < MP * MP; idx += kWG) {
            const int r = idx / MP, c = idx - r * MP;
            double v;
            if (r == k) v = (c == k) ? pinv : rowk[c] * pinv;
            else if (c == k) v = -colk[r] * pinv;
            else v = a[r * LD + c] - colk[r] * rowk[c] * pinv;
            a[r * LD + c] = v;
        }
        __syncthreads();
    }
    double *W = blk + ((size_t)i * NB + B) * MP * MP;
    for (int idx = threadIdx.x; idx < MP * MP; idx += kWG) {
        const int r = idx / MP, c = idx - r * MP;
        W[idx] = (r < n && c < n) ? a[r * LD + c] : 0.0;
    }
    if (threadIdx.x == 0 && bad) atomicAdd(&st->bad_blocks, 1);
}

// ---------------------------------------------------------------------------
// W_i = (-Q_ii)^{-1} by blocked Gauss-Jordan elimination with FP64 MFMA, one
// level per workgroup, the whole block in LDS.  For each 16-wide panel k:
//   D^{-1}     inverse of the 16x16 diagonal tile (one wave, VALU, computed
//              during the previous panel's trailing update)
//   R          = D^{-1} A[k, j]              row panel, j != k      (MFMA)
//   A[i, j]   -= A[i, k] R[k, j]             trailing update, i, j != k (MFMA)
//   A[i, k]    = -A[i, k] D^{-1},  A[k, k] = D^{-1}   column panel  (MFMA)
// which is the unblocked elimination of k_invert regrouped by panels, so it
// needs no pivoting for the same reason; a diagonal-tile pivot that is not
// clearly positive relative to the original diagonal marks the block singular.
// v_mfma_f64_16x16x4f64 lane layout: A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k, D[i][j] in register i / 4 of lane j + 16 (i % 4).
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ inline d4_t mfma16x16x4(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Waves per workgroup of the MFMA inverse.  The block fills the LDS at
// MP = 128, so one workgroup runs per CU; 16 waves (4 per SIMD) let the MFMA
// chains of different tiles overlap (1.3x over 4 waves, same arithmetic per
// tile, so bitwise the same inverse).  At MP = 64 several workgroups share
// a CU and 8 waves gain 3 %; more waves cost occupancy.
__host__ __device__ constexpr int inv_waves(int MP) { return MP >= 128 ? 16 : MP >= 64 ? 8 : 4; }

// Row KG (lanes 16 KG .. 16 KG + 15) of x, copied into every row of 16
// lanes: a swap of the wave's halves, then of neighbouring rows
// (v_permlane32_swap, v_permlane16_swap; each returns both swapped operands).
template <int KG>
__device__ __forceinline__ unsigned row_bcast(unsigned x) {
    const auto h = __builtin_amdgcn_permlane32_swap(x, x, false, false);   // rows 0 1 0 1 | 2 3 2 3
    const unsigned y = h[KG >> 1];
    const auto r = __builtin_amdgcn_permlane16_swap(y, y, false, false);   // rows a a b b | c c d d
    return r[KG & 1];
}

// Gauss-Jordan steps K .. 15 of invert_diag_tile (K a constant: the lane
// broadcasts take it as an immediate).
template <int K>
__device__ __forceinline__ void gj_steps(double (&t)[4], int c, int g, double &piv) {
    if constexpr (K < 16) {
        constexpr int kg = K & 3, kv = K >> 2;    // row K: lanes of group kg, register kv
        // (K, c): row kg of the wave, copied into every row of 16 lanes
        const double row = __hiloint2double((int)row_bcast<kg>((unsigned)__double2hiint(t[kv])),
                                            (int)row_bcast<kg>((unsigned)__double2loint(t[kv])));
        // (r, K): lane K of the lane's own row of 16 (DPP row_newbcast)
        double col[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
            col[v] = __hiloint2double(
                __builtin_amdgcn_mov_dpp(__double2hiint(t[v]), 0x150 + K, 0xF, 0xF, false),
                __builtin_amdgcn_mov_dpp(__double2loint(t[v]), 0x150 + K, 0xF, 0xF, false));
        // (K, K), read from its lane into every lane
        const double pk = __hiloint2double(
            __builtin_amdgcn_readlane(__double2hiint(t[kv]), 16 * kg + K),
            __builtin_amdgcn_readlane(__double2loint(t[kv]), 16 * kg + K));
        const double pinv = 1.0 / pk;
        const double rs = (c == K ? 1.0 : row) * pinv;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double gen = (c == K ? 0.0 : t[v]) - col[v] * rs;
            t[v] = (g + 4 * v == K) ? rs : gen;
        }
        piv = (c == K) ? pk : piv;   // lane c keeps the pivot of step c
        gj_steps<K + 1>(t, c, g, piv);
    }
}

// Inverse of the 16 x 16 diagonal tile kb of the block a (row stride LD, in
// LDS) into dst (row stride DL), by one wave, in registers: lane (g, c)
// holds column c = lane % 16 of rows g + 4 v, g = lane / 16.  Each
// Gauss-Jordan step copies its pivot row to every row of 16 lanes and its
// pivot column across each row of 16 lanes (register-to-register lane
// moves), reads the pivot from its lane, and scales by one reciprocal of it;
// every lane runs the same instructions (selects, no branches).  A pivot
// not above 1e-13 times the original diagonal entry, or not finite, sets
// *bad (lane c checks the pivot of step c).
template <int LD, int DL>
__device__ __forceinline__ void invert_diag_tile(const double *a, const double *dorig, int kb,
                                                 double *dst, int *bad) {
    const int lane = threadIdx.x & 63;
    const int k0 = 16 * kb;
    const int c = lane & 15, g = lane >> 4;
    double t[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = a[(k0 + g + 4 * v) * LD + k0 + c];
    double piv = 0.0;
    gj_steps<0>(t, c, g, piv);
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[(g + 4 * v) * DL + c] = t[v];
    if (!(piv > 1e-13 * dorig[k0 + c]) || !isfinite(piv)) *bad = 1;
}

// The blocked elimination of k_invert_mfma on a block a (row stride LD, in
// LDS or, for the large blocks, global memory), in place, by the whole
// workgroup of NW waves: dorig holds the block's original diagonal (for the
// pivot checks), dinv two 16 x 16 tiles of LDS, *bad is set on a pivot
// that is not clearly positive.
template <int MP, int NW, int LD>
__device__ __forceinline__ void gj_blocked(double *a, const double *dorig,
                                           double (*dinv)[16 * 17], int *bad) {
    constexpr int NT = MP / 16;     // panels
    constexpr int DL = 17;          // stride of the 16x16 tile
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lq = lane >> 4;   // lane's row/column in a 16-wide tile, quarter
    if (wave == 0) invert_diag_tile<LD, DL>(a, dorig, 0, dinv[0], bad);
    __syncthreads();
    for (int kb = 0; kb < NT; ++kb) {
        const int k0 = 16 * kb;
        const double *dcur = dinv[kb & 1];
        // row panel: R = D^{-1} A[k, j]
        for (int jb = wave; jb < NT; jb += NW) {
            if (jb == kb) continue;
            const int j0 = 16 * jb;
            d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const double av = dcur[lr * DL + 4 * s4 + lq];
                const double bv = a[(k0 + 4 * s4 + lq) * LD + j0 + lr];
                acc = mfma16x16x4(av, bv, acc);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) a[(k0 + lq + 4 * v) * LD + j0 + lr] = acc[v];
        }
        __syncthreads();
        // trailing update: A[i, j] += (-A[i, k]) R[k, j] over the tiles
        // outside row and column kb.  Lookahead: wave 0 updates the next
        // panel's diagonal tile and inverts it while the other waves update
        // the remaining tiles (the column panel below leaves that tile
        // alone).  Each wave reads its next tile's operands from LDS before
        // the current tile's MFMAs (tiles are disjoint and panel kb is not
        // written here).
        {
            constexpr int NTR = (NT - 1) * (NT - 1);
            const bool ahead = kb + 1 < NT;
            const int tl = kb * (NT - 1) + kb;   // the next diagonal tile among the NTR
            auto tile_at = [&](int t, int &i0, int &j0) {
                int ib = t / (NT - 1), jb = t - ib * (NT - 1);
                ib += ib >= kb;
                jb += jb >= kb;
                i0 = 16 * ib;
                j0 = 16 * jb;
            };
            auto fetch = [&](int i0, int j0, d4_t &acc, double *av, double *bv) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] = a[(i0 + lq + 4 * v) * LD + j0 + lr];
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    av[s4] = -a[(i0 + lr) * LD + k0 + 4 * s4 + lq];
                    bv[s4] = a[(k0 + 4 * s4 + lq) * LD + j0 + lr];
                }
            };
            auto update = [&](int i0, int j0, d4_t acc, const double *av, const double *bv) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) acc = mfma16x16x4(av[s4], bv[s4], acc);
#pragma unroll
                for (int v = 0; v < 4; ++v) a[(i0 + lq + 4 * v) * LD + j0 + lr] = acc[v];
            };
            // the tiles this wave updates: u = u0, u0 + du, ... < nu, which
            // skip the lookahead tile when there is one
            const int nu = ahead ? NTR - 1 : NTR;
            const int u0 = ahead ? wave - 1 : wave, du = ahead ? NW - 1 : NW;
            auto tile_of = [&](int u) { return (ahead && u >= tl) ? u + 1 : u; };
            if (ahead && wave == 0) {
                int i0, j0;
                d4_t acc;
                double av[4], bv[4];
                tile_at(tl, i0, j0);
                fetch(i0, j0, acc, av, bv);
                update(i0, j0, acc, av, bv);
                invert_diag_tile<LD, DL>(a, dorig, kb + 1, dinv[(kb + 1) & 1], bad);
            } else {
                int u = u0, i0 = 0, j0 = 0;
                d4_t acc;
                double av[4], bv[4];
                if (u < nu) {
                    tile_at(tile_of(u), i0, j0);
                    fetch(i0, j0, acc, av, bv);
                }
                while (u < nu) {
                    const int un = u + du;
                    int i0n = 0, j0n = 0;
                    // defined also when there is no next tile (then unused)
                    d4_t accn = {0.0, 0.0, 0.0, 0.0};
                    double avn[4] = {0.0, 0.0, 0.0, 0.0}, bvn[4] = {0.0, 0.0, 0.0, 0.0};
                    if (un < nu) {
                        tile_at(tile_of(un), i0n, j0n);
                        fetch(i0n, j0n, accn, avn, bvn);
                    }
                    update(i0, j0, acc, av, bv);
                    u = un;
                    i0 = i0n;
                    j0 = j0n;
                    acc = accn;
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        av[s4] = avn[s4];
                        bv[s4] = bvn[s4];
                    }
                }
            }
        }
        __syncthreads();
        // column panel: A[i, k] = -A[i, k] D^{-1};  A[k, k] = D^{-1}
        for (int ib = wave; ib < NT; ib += NW) {
            const int i0 = 16 * ib;
            d4_t acc = {0.0, 0.0, 0.0, 0.0};
            if (ib == kb) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] = dcur[(lq + 4 * v) * DL + lr];
            } else {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    const double av = -a[(i0 + lr) * LD + k0 + 4 * s4 + lq];
                    const double bv = dcur[(4 * s4 + lq) * DL + lr];
                    acc = mfma16x16x4(av, bv, acc);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) a[(i0 + lq + 4 * v) * LD + k0 + lr] = acc[v];
        }
        __syncthreads();
    }
}

// GLOBAL (blocks above 128, whose 512 KB do not fit in LDS): the same
// elimination in place in the output block W_i, in global memory (the
// workgroup's barriers order its accesses; the block stays in L2).
template <int MP, int NW = inv_waves(MP), bool GLOBAL = (MP > 128)>   // NW: waves per workgroup
__global__ __launch_bounds__(64 * NW) void k_invert_mfma(const double *diag, const int *sizes,
                                                      double *blk, int NB, int B, DevState *st) {
    constexpr int LD = GLOBAL ? MP : MP + 2;   // row stride of the working block (doubles)
    constexpr int DL = 17;          // stride of the 16x16 tile
    static_assert(NW >= 2, "the lookahead wave needs partners for the trailing update");
    __shared__ double a_lds[GLOBAL ? 1 : MP * LD];
    __shared__ double dinv[2][16 * DL];   // D^{-1} of this panel and of the next
    __shared__ double dorig[MP];
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int i = blockIdx.x;
    const int n = sizes[i];
    const double *Q = diag + (size_t)i * MP * MP;
    double *W = blk + ((size_t)i * NB + B) * MP * MP;
    double *a;
    if constexpr (GLOBAL)
        a = W;
    else
        a = a_lds;
    if (tid == 0) bad = 0;
    if constexpr (GLOBAL) {
        for (int idx = tid; idx < MP * MP; idx += 64 * NW) {
            const int r = idx / MP, c = idx - r * MP;
            const double v = (r < n && c < n) ? -Q[idx] : (r == c ? 1.0 : 0.0);
            a[idx] = v;
            if (r == c) dorig[r] = v;
        }
    } else {
        // every load of the thread's share issued before the first LDS store
        // (the block is stored padded to MP x MP, so all of it is readable)
        constexpr int PER = MP * MP / (64 * NW);
        double q[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) q[u] = Q[tid + u * 64 * NW];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = tid + u * 64 * NW;
            const int r = idx / MP, c = idx - r * MP;
            double v;
            if (r < n && c < n) v = -q[u];
            else v = (r == c) ? 1.0 : 0.0;
            a[r * LD + c] = v;
            if (r == c) dorig[r] = v;
        }
    }
    __syncthreads();
    gj_blocked<MP, NW, LD>(a, dorig, dinv, &bad);
    if constexpr (GLOBAL) {
        // the inverse is in place: clear the padding
        for (int idx = tid; idx < MP * MP; idx += 64 * NW) {
            const int r = idx / MP, c = idx - r * MP;
            if (!(r < n && c < n)) W[idx] = 0.0;
        }
    } else {
#pragma unroll
        for (int u = 0; u < MP * MP / (64 * NW); ++u) {
            const int idx = tid + u * 64 * NW;
            const int r = idx / MP, c = idx - r * MP;
            W[idx] = (r < n && c < n) ? a[r * LD + c] : 0.0;
        }
    }
    if (tid == 0 && bad) atomicAdd(&st->bad_blocks, 1);
}

// ---------------------------------------------------------------------------
// host-side helpers shared by the launcher files
// ---------------------------------------------------------------------------
// Levels per workgroup of variant v's tile for block size MP.
template <typename T, int MP>
static int lpw_mp(int v) {
    switch (variant_rg(MP, v)) {
        case 1: return Tile<T, MP, 1>::LPW;
        case 2: return Tile<T, MP, 2>::LPW;
        case 4: return Tile<T, MP, 4>::LPW;
        default: return Tile<T, MP, 8>::LPW;
    }
}

template <typename T>
static int lpw_of(int MP, int v) {
    switch (MP) {
        case 8: return lpw_mp<T, 8>(v);
        case 16: return lpw_mp<T, 16>(v);
        case 32: return lpw_mp<T, 32>(v);
        case 64: return lpw_mp<T, 64>(v);
        case 128: return lpw_mp<T, 128>(v);
        case 256: return lpw_mp<T, 256>(v);
    }
    return 1;
}

// Launch through hipExtLaunchKernel when the dispatch is timed, so that the
// events carry the kernel's own start and end.
template <typename K, typename... Args>
static void launch_timed(K kernel, int groups, hipStream_t s, LaunchTimer t, Args... args) {
    if (t.start || t.stop)
        hipExtLaunchKernelGGL(kernel, dim3(groups), dim3(kWG), 0, s, t.start, t.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, dim3(groups), dim3(kWG), 0, s, args...);
}

// Per-precision entry points, instantiated in their own files.
template <typename T>
hipError_t sweep_phase_t(int MP, int b, bool phase_b, int variant, const SweepLaunch &a,
                         hipStream_t s, LaunchTimer t);
template <typename T>
int flow_dispatch_t(int MP, int b, bool launch, int variant, const FlowLaunch *f, hipStream_t s,
                    hipError_t *err);
hipError_t launch_flow_reset(unsigned *flags, int n, hipStream_t s);

}  // namespace stc
