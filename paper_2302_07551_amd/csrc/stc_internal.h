// Internal declarations shared by the host runtime (stc_runtime.cpp) and the
// device kernels (stc_kernels.hip) of the staircase solver library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/stc.h"

namespace stc {

// Device-side solver state of one chain (lives in the arena).
// Ring slots are indexed by the sweep number s modulo kRing:
//   inv_sigma[s] = 1 / e^T W_s   (W_s: unnormalised output of sweep s,
//                                 W_0 = the loaded start vector; slot -1
//                                 holds 1 / e^T W_0 too, the scale of sweep 1)
//   diff[s]      = ||x^(s) - x^(s-1)||_1 with x^(s) = W_s * inv_sigma[s]
constexpr int kRing = 4096;
constexpr int kRingMask = kRing - 1;

struct DevState {
    double inv_sigma[kRing];
    double diff[kRing];
    double residual;          // last residual evaluation
    double x_sum;             // e^T of the last loaded vector
    int stop_flag;            // 1: no further sweep may change the iterate
    int status;               // 0 ok, 1 degenerate sum, 2 bad start vector
    long long stop_sweep;     // sweep whose change met the device test
    long long last_sweep;     // last sweep whose phase B finished
    int bad_blocks;           // singular diagonal blocks found by the inverse
    int pad_;
    long long test_after;     // changes of sweeps <= test_after are neither recorded
                              // nor tested (set at a precision switch: their
                              // iterates were overwritten after the FP32 stop)
    long long burst_base;     // batched sweeps: the first sweep of the burst in
                              // progress (sweep j of the burst is burst_base + j)
};

enum DevStatus { kDevOk = 0, kDevDegenerate = 1, kDevBadStart = 2, kDevTimeout = 3 };

// One launch of a half-sweep (phase A or phase B) of one chain.
struct SweepLaunch {
    const void *blk;      // T [L][2b+1][MP][MP] gather-oriented blocks
    const void *w_old;    // T [L][MP]  W_{s-1}
    const void *w_d1;     // T [L][MP]  W_{s-2}  (change of sweep s-2)
    const void *w_d2;     // T [L][MP]  W_{s-3}
    void *w_new;          // T [L][MP]  W_s
    double *part_sum;     // per-workgroup partial e^T W_s
    double *part_diff;    // per-workgroup partial change
    DevState *st;
    int L;
    int parity;           // first level of this phase
    int slot0;            // first partial slot used by this launch
    int nslots;           // total slots of both phases
    long long s;          // sweep being produced (>= 1)
    // Phase B only: one extra workgroup reduces the partials of sweep s-1 and
    // records them (instead of a finalize launch between the sweeps).
    int fold;
    int prev_nslots;
    const double *prev_sum;
    const double *prev_diff;
    double tol;           // device change test applied when recording
};

// Launch variants of the sweep kernels (picked per chain by the autotuner):
//   bit 0: 4 row groups per level instead of 8 (more levels per workgroup,
//          longer per-thread row streams)
//   bit 1: non-temporal block loads (streamed blocks bypass cache allocation,
//          so the iterate vectors stay cached; best once the blocks exceed
//          the last-level cache)
//   bit 2: a burst of sweeps runs as one persistent cooperative launch whose
//          blocks wait on their neighbours' progress flags instead of on
//          kernel boundaries (same per-level arithmetic and reductions, so the
//          same results bit for bit)
// The row groups per level follow the block size: blocks of 64 and more take
// 8 (bit 0 clear) or 4 (bit 0 set); blocks of 16 and 32 take MP / 8 or
// MP / 16, so that a thread streams 8 or 16 rows of each block between two
// workgroup barriers instead of 1 to 4.  Blocks of 8 take 1 row group (bit 0
// clear: a thread streams all 8 rows) or 4 (bit 0 set: a team's load then
// covers 4 whole rows, 128 contiguous bytes in FP32, 256 in FP64, instead of
// 32 or 64 bytes of each of 32 or 16 levels).  Bit 3 is internal: the fixed
// 8-row-group tile of the sparse kernel.
constexpr int kVariants = 8;
constexpr int kMaxBandwidth = 4;   // block bandwidth b of the generators taken
constexpr int kEllGeometry = 8;
__host__ __device__ constexpr int variant_rg(int MP, int v) {
    return (v & kEllGeometry) ? 8
           : MP >= 64         ? ((v & 1) ? 4 : 8)
           : MP == 8          ? ((v & 1) ? 4 : 1)
           : (v & 1)          ? MP / 16
                              : MP / 8;
}
__host__ __device__ constexpr bool variant_nt(int v) { return (v & 2) != 0; }
__host__ __device__ constexpr bool variant_flow(int v) { return (v & 4) != 0; }

// A burst of n sweeps in one cooperative launch (launch variant bit 2).
// Blocks 0..G-1 each own a contiguous range of the groups of both phases and
// run every sweep of the burst, waiting only on the progress flags of the
// two neighbouring blocks; block G is the folder, which reduces each sweep's
// partials once all blocks have finished it and records the sweep.
struct FlowLaunch {
    const void *blk;
    void *w[4];               // iterates W_s in rotation: buffer s % 4
    double *part_sum;         // [2][nparts] partials, by sweep parity
    double *part_diff;
    int nparts;
    DevState *st;
    int L;
    int parity_a;             // first level of phase A
    int groups_a, groups_b;   // groups of each phase
    int G;                    // streaming blocks (the folder is block G)
    unsigned *flags;          // [2 G + 2]: phase A done [G], phase B done [G], folded,
                              // abort
    long long s0;             // sweeps s0+1 .. s0+n
    int n;
    double tol;
    long long timeout_ticks;  // a wait longer than this (wall clock) aborts
};

// One sparse off-diagonal block, stored by rounds of slot quads.  Column j
// holds its nonzeros in row order, in q_j = ceil(nnz_j / 4) quads (the last
// one padded with value 0, row 0).  Round t holds quad t of every column with
// q_j > t, in column order and with no gaps: the quad of column j sits at
// quad position base_t + rank_t(j), rank_t(j) = #{j' < j : q_j' > t}, that
// is at slot off + 4 (base_t + rank_t(j)) in the value and row-index pools.
// The row-index pool also holds, from byte meta (a multiple of 4), the
// block's q_j (MP bytes) and then base_0 .. base_Kq (Kq + 1 unsigned
// shorts, base_0 = 0).  Kq = max q_j rounds; 4 base_Kq slots in all.
struct EllEntry {
    long long off;
    int Kq;
    int meta;
};

// The off-diagonal entries of one level of a generator of any block pattern
// (column-major ELL in slot quads, like EllEntry, with 32-bit indices into
// the padded iterate, level * MP + state).  Column j of the level holds Kn
// "near" slots, whose sources lie in the adjacent levels i - 1 and i + 1
// (read fresh by phase B), then Kf "far" slots from every other level (read
// from the previous iterate by both phases); Kn and Kf are multiples of 4.
// Near slot k = 4 kq + t of column j sits at off + (kq MP + j) 4 + t, far
// slot k at off + Kn MP + (kq MP + j) 4 + t.  Padding slots hold the value 0
// and the index of a state that every read of that slot finds written.
struct GenEntry {
    long long off;
    int Kn, Kf;
};

// One chain of a batched (multi-chain) launch, as the device reads it.  The
// blocks and iterate buffers are those of the chain's current precision
// stage; its sweep number is DevState::last_sweep + 1.
struct ChainDesc {
    const void *blk;
    void *w[4];           // rotation: W_s lives in w[s % 4]
    double *part_sum;
    double *part_diff;
    DevState *st;
    int L, MP, parity_a;  // levels, padded block size, first phase-A level
    int groups_a, groups_b;
    int nparts;           // partial slots per sweep parity: sweep s uses
                          // part_sum[(s & 1) * nparts ..]
    double tol;           // device change test for this chain (<= 0: off)
};

// One workgroup's work in a batched half-sweep: groups group .. group +
// count - 1 of chain c, one after the other (each still writes its own
// partial slot, so the number of groups per item does not change results).
// group < 0 (phase A only, listed first): the reduction of the chain's
// previous sweep, folded into this launch instead of a launch of its own.
struct WorkItem {
    int chain;
    int group;
    int count;
};

// One chain's state as stc_batch_query reports it.
struct QueryRow {
    long long sweeps;       // sweep of the current iterate (the stop sweep once stopped)
    long long last_sweep;   // last sweep whose phase B finished
    double diff;            // latest change known for certain (+inf if none)
    int stopped;
    int status;             // DevStatus
};

// Largest number of per-group partial slots of a sweep that the extra
// workgroup of phase B reduces; above it a finalize launch follows every
// sweep.  The fold's loads run U slots ahead, so 65536 slots take a few
// microseconds, while a phase of that many groups streams for hundreds.
constexpr int kFoldSlots = 65536;

// Host-visible launchers (stc_kernels.hip).  Each returns a hipError_t.
int supported_mp(int m);   // padded block size for m, or 0
int variant_count();
int phase_groups(int precision_bytes, int MP, int L, int parity, int variant);
// The sweep launchers take an optional pair of events attached to the
// dispatch itself (hipExtLaunchKernel): they time the kernel alone, without
// the markers a separate hipEventRecord adds to the stream.
struct LaunchTimer {
    hipEvent_t start = nullptr, stop = nullptr;
};
hipError_t launch_sweep_phase(int precision_bytes, int MP, int b, bool phase_b, int variant,
                              const SweepLaunch &a, hipStream_t stream,
                              LaunchTimer t = LaunchTimer());
hipError_t launch_sweep_phase_ell(int precision_bytes, int MP, int b, bool phase_b,
                                  const SweepLaunch &a, const EllEntry *tab, const void *val,
                                  const unsigned char *idx, hipStream_t stream,
                                  LaunchTimer t = LaunchTimer());
// Generators of any block pattern (stc_general.hip): the sweep phases and
// the residual, over the diagonal blocks (inverse W_i in blk, Q_ii in diag)
// and the per-level GenEntry table.
// nt: non-temporal loads of the stored blocks and entries.  Blocks above
// kMaxSmallMP take the large-block kernels, which need rbuf: a scratch
// vector of L x MP elements of the sweep's type.
hipError_t launch_sweep_phase_gen(int precision_bytes, int MP, bool phase_b, bool nt,
                                  const SweepLaunch &a, const GenEntry *tab, const void *val,
                                  const int *idx, void *rbuf, hipStream_t stream,
                                  LaunchTimer t = LaunchTimer());
hipError_t launch_residual_gen(int precision_bytes, int MP, const double *diag64,
                               const GenEntry *tab, const double *val64, const int *idx,
                               const void *w, int L, DevState *st, long long slot, double *part,
                               hipStream_t stream, double *out = nullptr);
// Most blocks of a persistent sweep kernel that can be resident at once
// (0 if the variant has no persistent form for these sizes).
int flow_resident_blocks(int precision_bytes, int MP, int b, int variant);
hipError_t launch_sweep_flow(int precision_bytes, int MP, int b, int variant, const FlowLaunch &f,
                             hipStream_t stream);
hipError_t launch_batch_query(DevState *const *states, int n, QueryRow *out, hipStream_t stream);
hipError_t launch_finalize_sweep(const double *part_sum, const double *part_diff, int nslots,
                                 DevState *st, long long s, double tol, hipStream_t stream);
hipError_t launch_invert(int MP, int b, const double *diag, const int *sizes, double *blk,
                         int L, DevState *st, hipStream_t stream);
hipError_t launch_cast_blocks(const double *src, float *dst, size_t n, hipStream_t stream);
hipError_t launch_load(int precision_bytes, int MP, const double *x, const long long *off,
                       const int *sizes, int L, void *w0, double *part, int nparts,
                       DevState *st, int state_slot, hipStream_t stream);
hipError_t launch_store(int precision_bytes, int MP, const void *w, const long long *off,
                        const int *sizes, int L, DevState *st, long long slot, double *x,
                        hipStream_t stream);
// ||Q^T w||_1 into DevState::residual, or into *out (device) when out is set.
hipError_t launch_residual(int precision_bytes, int MP, int b, const double *blk64,
                           const double *diag64, const void *w, int L, DevState *st,
                           long long slot, double *part, hipStream_t stream,
                           double *out = nullptr);
// Krylov acceleration (stc_krylov.hip): vectors are FP64 padded [L][MP].
constexpr int kDotGroups = 128;     // chunks of a vector per partial dot
constexpr int kMaxRestart = 256;    // largest GMRES restart length
hipError_t launch_kstate_init(DevState *st, hipStream_t s);
// out[v] = V[v] . w for v < nv (w = nullptr: e^T V[v]; absdiff:
// ||V[v] - w||_1); norm: out[0] = sqrt(V[0] . w).  part holds G * nv doubles.
hipError_t launch_kdots(const double *V, size_t ld, int nv, const double *w, size_t n,
                        double *part, int G, double *out, bool norm, hipStream_t s,
                        bool absdiff = false);
// w += sign * sum_v h[v] V[v], h in device memory
hipError_t launch_kupdate(const double *V, size_t ld, int nv, const double *h, double sign,
                          double *w, size_t n, hipStream_t s);
hipError_t launch_kaxpby(double a, const double *x, double b, const double *y, double *out,
                         size_t n, hipStream_t s);
// out = x / sdev[0]
hipError_t launch_kscale(const double *x, const double *sdev, double *out, size_t n,
                         hipStream_t s);
// Sum the per-group residual partials into DevState::residual (or *out).
hipError_t launch_reduce_residual(const double *part, int n, DevState *st, hipStream_t stream,
                                  double *out = nullptr);
hipError_t launch_diff(int precision_bytes, int MP, int variant, const void *w,
                       const void *w_prev, int L, int parity_a, DevState *st, long long k,
                       double *part, hipStream_t stream, double tol);
hipError_t launch_widen(const float *src, double *dst, size_t n, hipStream_t stream);
hipError_t launch_reset_state(DevState *st, hipStream_t stream);
hipError_t launch_rearm(DevState *st, long long k, hipStream_t stream);
// One batched half-sweep launch of the chains of one padded block size:
// variant bits 0 (row groups) and 1 (non-temporal loads) as for one chain.
// j: the sweep's index in its burst (sweep burst_base + j of each chain).
hipError_t launch_batch_phase(int precision_bytes, int b, int MP, bool phase_b, int variant,
                              int grid, const ChainDesc *chains, const WorkItem *items,
                              const int *nitems, int j, hipStream_t stream);
// Finalize of sweep burst_base + j of chains[range[0] ..][0 .. range[1] - 1]
// (range on the device); grid: at least the largest range[1] the launch may
// see.
hipError_t launch_batch_finalize(int grid, const ChainDesc *chains, const int *range, int j,
                                 hipStream_t stream);
// Start of a burst for the same chains: burst_base = last_sweep + 1.
hipError_t launch_batch_begin(int grid, const ChainDesc *chains, const int *range,
                              hipStream_t stream);
int reduce_groups(int MP, int L);

// Largest padded block size of the one-workgroup-per-level kernels; the
// padded sizes 512, 1024 and 2048 (generators of any block pattern only)
// take the large-block kernels of stc_big.hip.
constexpr int kMaxSmallMP = 256;
constexpr int kMaxMP = 2048;
// Large blocks: column slices per level of a sweep phase (one partial slot
// each) and of the residual.
int big_slices(int precision_bytes, int MP);
int big_residual_slices(int MP);
// One phase of a large-block sweep: the gather launch, then the apply
// launch (with phase B's reduction workgroup when a.fold).
hipError_t launch_sweep_phase_big(int precision_bytes, int MP, bool phase_b, bool nt,
                                  const SweepLaunch &a, const GenEntry *tab, const void *val,
                                  const int *idx, void *rbuf, hipStream_t stream, LaunchTimer t);
// The change of sweep k in the apply kernel's slices, one partial per slice
// (phase A's gA slices, then phase B's gB).
hipError_t launch_diff_big_partials(int precision_bytes, int MP, const void *w, const void *w_prev,
                                    int parity_a, int gA, int gB, const DevState *st, long long k,
                                    double *part, hipStream_t stream);
// One sweep of Algorithm 1 on the large blocks: ceil(L / chunks) steps of a
// gather and an apply launch, step t taking the t-th level of every chunk
// (a.fold on the first step's apply); partials in slot i (MP / 64) + slice.
// Steps with few (level, slice) groups split each apply over row ranges into
// zpart (jgs_big_split_bytes(L, MP) bytes; null: never split) and add the
// ranges in a third launch.
hipError_t launch_sweep_jgs_big(int precision_bytes, int MP, bool nt, int chunks,
                                const SweepLaunch &a, const GenEntry *tab, const void *val,
                                const int *idx, void *rbuf, void *zpart, hipStream_t stream,
                                LaunchTimer t);
size_t jgs_big_split_bytes(int L, int MP);
// The change of sweep k in those slots (L (MP / 64) partials, levels in order).
hipError_t launch_diff_big_levels(int precision_bytes, int MP, const void *w, const void *w_prev,
                                  int L, const DevState *st, long long k, double *part,
                                  hipStream_t stream);
// W_i = (-Q_ii)^{-1} for the large blocks (blocked Gauss-Jordan over many
// workgroups per level), in place in blk (one MP x MP block per level), with
// scratch of big_invert_scratch_bytes(MP, L) bytes; singular levels are
// counted in st->bad_blocks.
size_t big_invert_scratch_bytes(int MP, int L);
hipError_t launch_invert_big(int MP, const double *diag, const int *sizes, double *blk, int L,
                             DevState *st, void *scratch, hipStream_t stream);
// ||Q^T x||_1 partials per (level, 64-column slice): groups = L x
// big_residual_slices(MP).
hipError_t launch_residual_big_partials(int precision_bytes, int MP, int groups,
                                        const double *diag, const GenEntry *tab, const double *val,
                                        const int *idx, const void *w, const DevState *st,
                                        long long slot, double *part, hipStream_t stream);

// Algorithm 1 (stc_jgs.hip): one sweep over `chunks` chunks of levels (the
// workgroups; plus the reduction workgroup of sweep s - 1 when a.fold), and
// the change of sweep k in its geometry, with the device stopping test.
hipError_t launch_sweep_jgs(int precision_bytes, int MP, int b, bool nt, int chunks,
                            const SweepLaunch &a, hipStream_t stream, LaunchTimer t);
// The same for a generator of any block pattern (stc_general.hip), padded
// blocks up to 256, from its per-level ELL; its partials follow the dense
// kernel's geometry, so launch_diff_jgs serves both (larger blocks:
// launch_sweep_jgs_big).
hipError_t launch_sweep_jgs_gen(int precision_bytes, int MP, bool nt, int chunks,
                                const SweepLaunch &a, const GenEntry *tab, const void *val,
                                const int *idx, hipStream_t stream, LaunchTimer t);
hipError_t launch_diff_jgs_partials(int precision_bytes, int MP, const void *w, const void *w_prev,
                                    int L, int chunks, const DevState *st, long long k,
                                    double *part, hipStream_t stream);
hipError_t launch_diff_jgs(int precision_bytes, int MP, const void *w, const void *w_prev, int L,
                           int chunks, DevState *st, long long k, double *part,
                           hipStream_t stream, double tol);

// Residual with caller-given device staging (stc_runtime.cpp), for the
// allocation-free entry point: bytes of staging the handle needs, the
// residual of x (device, compact) into out (device) on the handle's stream,
// and the library's error report (message for stc_last_error).
size_t residual_staging_bytes(const stc_handle *h);
stc_status residual_into(stc_handle *h, const double *x, double *out, int device, char *staging,
                         size_t staging_bytes);
stc_status report_error(stc_status s, const char *msg);

}  // namespace stc
