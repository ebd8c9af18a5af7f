/*
 * stc.h - C ABI of the block staircase-splitting solver for the stationary
 * vector of a continuous-time Markov chain on AMD Instinct MI355X (gfx950).
 *
 * Problem (eq. (1), section 1): given the generator Q of an irreducible chain
 * (off-diagonal rates >= 0, every row sums to 0), find pi with
 *     Q^T pi = 0,   pi >= 0,   e^T pi = 1.
 * Method (section 2): the normalised power-type iteration of eq. (mainsch)
 * for the regular splitting Q^T = M - N in which M is a stair matrix (type 1
 * or 2), implemented as in Algorithm 2.  One sweep has two parallel steps:
 * "phase A" solves the diagonal-only block rows independently; "phase B"
 * solves the stair rows from the freshly computed neighbours; then the sweep
 * normalises and measures ||x^(k+1) - x^(k)||_1.
 *
 * Levels: the states are grouped into L levels (the block partition of Q^T,
 * section 2), level i holding n_i <= m states; equal sizes with a smaller
 * last level is the paper's choice (section 3).  The generator is block
 * banded with block bandwidth b (1 = block tridiagonal / QBD, 2 = block
 * pentadiagonal).
 *
 * Conventions for every entry point:
 *   - Status codes only; nothing throws across this interface.  After any
 *     status other than STC_OK, stc_last_error() returns a message for the
 *     calling thread.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Host arrays passed in are only read during the call (the caller may
 *     free them afterwards) unless stated otherwise.
 *   - All device memory the library uses lives inside the caller's arena
 *     (stc_options.arena); the library allocates no device memory.
 *   - Vectors of length N = sum n_i are compact (level after level), FP64.
 *     Arguments marked "where" say whether a vector pointer is host memory
 *     (STC_MEM_HOST) or device memory on the handle's GPU (STC_MEM_DEVICE).
 */
#ifndef STC_H
#define STC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STC_OK = 0,
    STC_EINVAL = 1,      /* bad argument: sizes, null pointer, x0 with a negative,
                            non-finite or all-zero entry set, unsupported m      */
    STC_ENOTGEN = 2,     /* not a generator: negative or non-finite off-diagonal
                            rate, or a row that does not sum to 0               */
    STC_ESINGULAR = 3,   /* a diagonal block Q_ii is singular (states of a level
                            that can never leave it), so M is not invertible    */
    STC_EDEGENERATE = 4, /* a sweep produced e^T z <= 0 or a non-finite sum      */
    STC_EMAXIT = 5,      /* maxit sweeps without meeting tol; the last iterate
                            and its figures are still returned                  */
    STC_ENOMEM = 6,      /* the arena is smaller than stc_footprint_bytes()     */
    STC_EDEVICE = 7      /* a HIP runtime call or kernel launch failed           */
} stc_status;

enum { STC_FP64 = 0, STC_FP32 = 1, STC_MIXED = 2 };   /* stc_options.precision */
enum { STC_STOP_DIFF = 0, STC_STOP_RESIDUAL = 1 };     /* stc_options.stop      */
enum { STC_MEM_HOST = 0, STC_MEM_DEVICE = 1 };         /* "where" arguments     */
enum { STC_DENSE = 0, STC_SPARSE = 1 };                /* stc_options.format    */
enum { STC_ANY_PATTERN = -1 };                         /* stc_generator.b       */
enum { STC_STAIRCASE = 0, STC_JGS = 1 };               /* stc_options.method    */

/* The block generator (section 2 block partition), in one of two host forms.
 *
 * Dense blocks: blocks is an array [L][2b+1][m][m], row-major: blocks[i][d+b]
 * holds Q_{i,i+d} (rows = states of level i, columns = states of level i+d)
 * padded with zeros to m x m.  Slots with i+d outside [0, L) are ignored, as
 * is the padding.
 *
 * CSR (blocks NULL): the whole N x N generator, N = sum of the level sizes,
 * states numbered level by level, as compressed sparse rows.  Every entry
 * must lie in the block band (the levels of its row and column differ by at
 * most b) and no column may repeat within a row (STC_EINVAL otherwise);
 * explicit zeros are allowed.  Diagonal entries may be left out when
 * recompute_diagonal is 1.  Setup scatters the rows into blocks a range of
 * levels at a time, so it never holds a dense copy of the whole generator.
 *
 * Any block pattern (b = STC_ANY_PATTERN; CSR input and STC_SPARSE storage
 * only): the general localized case of section 2, where a level may couple to
 * any other level (block upper Hessenberg generators, state spaces ordered so
 * that transitions reach many levels away).  Every entry may lie anywhere; the
 * near entries (levels i - 1 and i + 1, the J_i of the stair rows in
 * Algorithm 2) are read fresh by phase B and all others from the previous
 * iterate.  L * padded m must stay below 2^31.  The block size may go up to
 * 2048, which covers the partitions of the experiments in section 3 (levels
 * of 256 to 2048 states); blocks padded to 512 and more are swept by column
 * slices of 64 states, one partial sum per slice.
 *
 * Either way the host arrays are only read during stc_footprint_bytes and
 * stc_setup, and the caller keeps ownership. */
typedef struct {
    int32_t L;                   /* levels, >= 2                                    */
    int32_t m;                   /* block size: max states per level, 1..128
                                    (1..2048 with b = STC_ANY_PATTERN)           */
    int32_t b;                   /* block bandwidth, 1..4 (1: QBD), or
                                    STC_ANY_PATTERN                                 */
    const int32_t *sizes;        /* [L] states per level n_i in 1..m; NULL = all m */
    const double *blocks;        /* dense blocks, see above; NULL = CSR input      */
    int32_t recompute_diagonal;  /* 1: diag(Q_ii) := -(row sum of its off-diagonal
                                    rates); 0: use the given diagonal, which must
                                    make every row sum to 0                        */
    const int64_t *csr_rowptr;   /* CSR input: [N+1], csr_rowptr[0] = 0, rising    */
    const int32_t *csr_col;      /* CSR input: [nnz] global column of each entry   */
    const double *csr_val;       /* CSR input: [nnz] rate of each entry            */
} stc_generator;

typedef struct {
    int32_t precision;    /* STC_FP64: FP64 blocks and sweeps.
                             STC_FP32: FP32 blocks and sweeps, FP64 sums.
                             STC_MIXED: FP32 sweeps until the change falls below
                             switch_tol, or stops falling (the FP32 rounding
                             floor: no new low over 4 readings taken every 32
                             sweeps or every check_every, if longer), then
                             FP64 sweeps to tol.                              */
    int32_t stair_type;   /* 1: M = M1 (phase A = even 0-based levels);
                             2: M = M2 (phase A = odd 0-based levels)         */
    int32_t stop;         /* STC_STOP_DIFF: ||x^(k) - x^(k-1)||_1 <= tol
                             (the stopping test of section 3);
                             STC_STOP_RESIDUAL: ||Q^T x^(k)||_1 <= tol        */
    int32_t check_every;  /* sweeps queued between host checks (>= 1).  The
                             change test runs on the device after every
                             sweep, so it stops at the exact sweep; the
                             residual test runs every check_every sweeps.    */
    double switch_tol;    /* STC_MIXED: FP32 -> FP64 switch threshold on the
                             change (<= 0: 1e-6)                              */
    void *stream;         /* hipStream_t used for every launch (NULL: null
                             stream)                                          */
    void *arena;          /* device memory owned by the caller, 256-byte
                             aligned, on the current device                  */
    size_t arena_bytes;   /* its size, >= stc_footprint_bytes()              */
    int32_t format;       /* device storage of the off-diagonal blocks swept:
                             STC_DENSE: dense m x m blocks;
                             STC_SPARSE: per block, its nonzeros grouped by
                             column and padded to the block's longest column
                             (values + 8-bit row indices), for sparse
                             (localized) generators; with b = STC_ANY_PATTERN
                             one ELL per level (values + 32-bit indices).
                             The inverse diagonal blocks are dense in both.
                             Batches take dense chains only.                  */
    int32_t krylov_restart; /* 0, or the longest restart length r (1..256) that
                             stc_solve_gmres may use: the footprint then holds
                             r + 3 FP64 vectors and small buffers for it     */
    int32_t krylov_keep_all; /* 0: stc_solve_gmres applies its safeguard (below);
                             1: every cycle is kept (textbook restarted GMRES,
                             no plain steps)                                   */
    int32_t method;       /* STC_STAIRCASE: the stair splitting (Algorithm 2).
                             STC_JGS: Algorithm 1 (section 2), the method the
                             paper compares against: the levels are cut into
                             jgs_chunks chunks of consecutive levels; a sweep
                             is block Jacobi across the chunks (a level reads
                             the previous iterate of every other chunk) and
                             block Gauss-Seidel inside each (the chunk's
                             levels in order, each reading the fresh values of
                             the chunk's earlier levels), then the same
                             normalisation and change.  jgs_chunks = 1 is
                             plain block Gauss-Seidel, jgs_chunks = L block
                             Jacobi.  Dense band storage, or STC_ANY_PATTERN
                             with m up to 2048 (each level's off-diagonal
                             entries read fresh or old by their source
                             level; above 256 a sweep is ceil(L / p) steps
                             of a few launches each, and the footprint adds
                             8 L m FP64 of scratch); no banded sparse
                             storage, no Krylov
                             workspace, not in batches; stair_type is
                             ignored; every other call works as for the
                             stair splitting.  */
    int32_t jgs_chunks;   /* STC_JGS: the number of chunks p, 1..L          */
} stc_options;

typedef struct {
    double residual_1;    /* ||Q^T pi||_1 of the returned pi, FP64            */
    double diff_1;        /* ||x^(k) - x^(k-1)||_1 at the returned sweep k    */
    int64_t iters;        /* k: sweeps that produced the returned pi          */
    int64_t iters_fp32;   /* of which in FP32 (STC_FP32 / STC_MIXED)          */
    int32_t status;       /* same value as the call's return code             */
} stc_result;

typedef struct stc_handle stc_handle;

/* Device bytes the handle needs for this generator and these options
 * (arena sub-allocation of every block copy, inverse, iterate and scratch).
 * Returns 0 for invalid arguments.  Used for admission decisions. */
size_t stc_footprint_bytes(const stc_generator *gen, const stc_options *opt);

/* Validate Q on the host, copy its blocks to the arena in the sweep's layout
 * and invert every diagonal block on the device: W_i = (-Q_ii)^{-1}, the
 * inverse of the diagonal block of M applied in both parallel steps of
 * Algorithm 2 (section 2).  FP32 copies are rounded from the FP64 ones.
 * Errors: STC_EINVAL, STC_ENOTGEN, STC_ESINGULAR, STC_ENOMEM, STC_EDEVICE.
 * On success *out owns no device memory of its own; it must be destroyed
 * before the arena is freed. */
stc_status stc_setup(const stc_generator *gen, const stc_options *opt, stc_handle **out);

/* ---- setup in two halves ----------------------------------------------
 * The same setup, split where the host work ends, for callers that overlap
 * setup with device work that another thread drives: stc_prepare does the
 * host half (validation of Q and the packing of its blocks in the sweep's
 * layout, on host threads) and makes no HIP call, so it may run on any
 * thread at any time; stc_setup_prepared does the device half (upload,
 * inverse of the diagonal blocks, FP32 copies, state) on opt->stream into
 * opt->arena.  stc_setup_prepared(stc_prepare(gen, opt), opt) gives the
 * handle stc_setup(gen, opt) gives, bit for bit.  Dense storage of
 * block-banded generators (b in 1..4) only: STC_EINVAL for other inputs,
 * which take stc_setup. */
typedef struct stc_prepared stc_prepared;

/* Host half.  opt's arena and stream are not used (the precision, format
 * and method are checked as by stc_setup).  *out owns a host copy of the
 * packed blocks (the device layout's size of blk64 and the diagonal blocks);
 * gen's arrays are not read after the call.  Errors: STC_EINVAL,
 * STC_ENOTGEN (the first bad level), STC_ENOMEM (host memory). */
stc_status stc_prepare(const stc_generator *gen, const stc_options *opt, stc_prepared **out);

/* Device half, on opt->stream into opt->arena (>= stc_footprint_bytes of the
 * same generator and options; opt may differ from stc_prepare's in its
 * precision, stop rule and the like, not in storage).  Returns when the
 * device work is done.  p stays owned by the caller.  Errors: STC_EINVAL,
 * STC_ENOMEM (arena), STC_ESINGULAR, STC_EDEVICE. */
stc_status stc_setup_prepared(const stc_prepared *p, const stc_options *opt, stc_handle **out);

/* Release what stc_prepare allocated (NULL is ignored). */
void stc_prepared_free(stc_prepared *p);

/* Algorithm 2 (section 2) with the stopping test of section 3: start from
 * x0 / e^T x0 (x0 NULL: e/N), sweep until the stop quantity is <= tol or
 * maxit sweeps were done, and write the last iterate to pi (length N).
 * x0 and pi are host or device memory per "where".  Returns STC_OK,
 * STC_EMAXIT (pi and res still filled), STC_EDEGENERATE, STC_EINVAL,
 * STC_EDEVICE.  res may be NULL. */
stc_status stc_solve(stc_handle *h, const double *x0, double tol, int64_t maxit,
                     double *pi, stc_result *res, int32_t where);

/* Krylov acceleration of the stair splitting: restarted GMRES(restart) on the
 * left-preconditioned singular system (I - M^{-1} N) x = 0, with M the stair
 * matrix of section 2, i.e. the splitting used as a preconditioner (the use
 * the Conclusions leave to future work).  Each cycle starts from the
 * normalised x, builds an orthonormal Krylov basis of M^{-1} A (M^{-1} N
 * applied by the sweep kernels without normalisation; classical
 * Gram-Schmidt, twice), takes the least-squares step and normalises again.
 * Cycles repeat until ||Q^T x||_1 <= tol or max_applies applications of
 * M^{-1} N.  Safeguard: on chains with strong drift the operator is far
 * from normal and short cycles can stall, so a cycle is kept only if it
 * lowers ||Q^T x||_1 per application by at least the square of the factor
 * the last block of plain steps achieved (before any plain block: by half
 * over the cycle); otherwise x stays and k plain normalised applications of
 * M^{-1} N follow, k = restart at first, doubled after each rejected cycle.
 * With opt.krylov_keep_all = 1 there is no safeguard: every cycle is kept,
 * as in textbook restarted GMRES, and a cycle whose sum is zero or not
 * finite ends the solve with STC_EDEGENERATE.
 * The Krylov vectors and the residual are always FP64.  An STC_FP64 handle
 * applies M^{-1} N in FP64; STC_FP32 and STC_MIXED handles apply it in FP32
 * (vectors rounded to FP32 for each application and widened back) until
 * ||Q^T x||_1 <= switch_tol or an FP32 cycle stalls, then in FP64 to tol;
 * res->iters_fp32 counts the FP32 applications.  x0 (NULL: e/N) is checked like stc_solve's;
 * pi receives the last normalised iterate.  res->iters counts the
 * applications, res->diff_1 the last cycle's change ||x_new - x||_1.
 * A cycle's x is normalised by its sum whatever its sign; a zero or
 * non-finite sum counts as a rejected cycle.  A cycle whose first Krylov
 * vector has zero or non-finite norm (T x = x to rounding) ends an FP32
 * stage, and in FP64 ends the solve with STC_EMAXIT if the residual is still
 * above tol.  Needs restart in 1..opt.krylov_restart (STC_EINVAL
 * otherwise).  Returns STC_OK, STC_EMAXIT (budget spent or stalled; pi and
 * res still filled), STC_EDEGENERATE (e^T x <= 0 after plain steps, or a
 * cycle without a usable sum under krylov_keep_all),
 * STC_EINVAL, STC_EDEVICE. */
stc_status stc_solve_gmres(stc_handle *h, const double *x0, int32_t restart, double tol,
                           int64_t max_applies, double *pi, stc_result *res, int32_t where);

/* One sweep of Algorithm 2 from x (normalised first): z = M^{-1} N x,
 * normalised, and *diff_1 = ||z - x/e^T x||_1.  In STC_FP32 / STC_MIXED the
 * sweep runs in FP32.  x and z are host or device memory per "where"; z may
 * not alias x. */
stc_status stc_step(stc_handle *h, const double *x, double *z, double *diff_1, int32_t where);

/* ||Q^T x||_1 in FP64 (eq. (1)), x as given (not normalised). */
stc_status stc_residual(stc_handle *h, const double *x, double *res_1, int32_t where);

/* Bytes of the static staging array of stc_residual_noalloc on each GPU. */
#define STC_NOALLOC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * residual of stc_residual, with the same value bit for bit, that allocates
 * nothing.  x: device memory, N FP64 (compact, as given, not normalised);
 * res_1: device memory, one FP64, written by the last kernel.  The calls are
 * enqueued on the handle's stream with no synchronisation and no host copy;
 * the handle's device must be current.  The padded copy of x and the
 * per-group partial sums are staged in a static device array of
 * STC_NOALLOC_SCRATCH_BYTES on each GPU (held until the process ends), which
 * every call on that GPU shares: calls that overlap on one GPU (other streams
 * or threads) race.  Every staged byte is written before it is read, so
 * nothing needs clearing between calls.  Also records e^T x in the handle's
 * state, as stc_residual does.  Returns STC_EINVAL for a null argument, a
 * device other than the handle's, or a handle whose staging (8 L m_pad bytes
 * plus its partial sums, m_pad the padded block size) exceeds the array;
 * STC_EDEVICE if a launch fails. */
stc_status stc_residual_noalloc(stc_handle *h, const double *x, double *res_1);

/* Device-resident sweeps: run nsweeps sweeps of Algorithm 2 on the handle's
 * current iterate without host synchronisation (the iterate is the one left by
 * the previous stc_solve / stc_step / stc_load on this handle).  diffs (host,
 * may be NULL) receives the change of every sweep but the last, after an
 * implicit synchronisation. */
stc_status stc_sweeps(stc_handle *h, int64_t nsweeps, double *diffs);

/* Measurement form of stc_sweeps: the same sweeps, each phase launched with
 * a start and a stop event attached to its dispatch (hipExtLaunchKernel), so
 * the phase times are the kernels' own (for blocks padded to 512 and more a
 * phase is two launches, its gather and its apply: the start event goes with
 * the first and the stop event with the second, so the time covers both).
 * Returns the mean device time of the
 * phase-A launch, of the phase-B launch, of the finalize work per sweep (the
 * per-sweep finalize launches of long chains plus the flush that ends the
 * burst, spread over the sweeps), and the mean wall time of a whole sweep
 * between events recorded around the burst, in milliseconds (any pointer may
 * be NULL). */
stc_status stc_profile_sweeps(stc_handle *h, int64_t nsweeps, double *ms_phase_a,
                              double *ms_phase_b, double *ms_finalize, double *ms_sweep);

/* Launch variants of the sweep kernels.  A variant fixes the thread shape of
 * a level (8 or 4 row groups per block) and whether block streams use
 * non-temporal loads; the result of a sweep does not depend on it beyond
 * rounding order.  stage is STC_FP64 or STC_FP32 (the precision of the
 * sweeps the variant applies to).  setup picks a default from the block
 * size and the bytes of the blocks.  For a generator of any pattern
 * (STC_ANY_PATTERN) only bit 1 applies: non-temporal loads of the inverse
 * blocks and entries, the default once they exceed the 256 MB last-level
 * cache (below it they stay cached from sweep to sweep); the banded sparse
 * kernel has no variants. */
int32_t stc_variant_count(void);
stc_status stc_set_variant(stc_handle *h, int32_t stage, int32_t variant);
stc_status stc_get_variant(stc_handle *h, int32_t stage, int32_t *variant);

/* Autotuner: for each precision stage the handle sweeps in, time every
 * variant over trial_sweeps sweeps of this chain (after 3 warm-up sweeps,
 * from e/N) and keep the fastest; a persistent variant is kept only if it
 * beats the fastest per-phase variant by more than 2 %.  Returns the mean
 * sweep times of the kept variants (ms, may be NULL).  It moves the
 * handle's iterate: the handle is left loaded with e/N, so call it before
 * stc_load / stc_sweeps (stc_solve reloads anyway). */
stc_status stc_autotune(stc_handle *h, int32_t trial_sweeps, double *ms_fp64, double *ms_fp32);

/* Algorithmic HBM bytes of one launch of phase A and of phase B for this
 * handle's current precision: every stored block the phase reads once, the
 * vector segments it reads once and the segments it writes once. */
stc_status stc_phase_bytes(stc_handle *h, double *bytes_phase_a, double *bytes_phase_b);

/* Set the handle's current iterate to x / e^T x (host or device memory). */
stc_status stc_load(stc_handle *h, const double *x, int32_t where);

/* Per-handle figures after stc_sweeps or batched sweeps: the sweep of the
 * current iterate (the stopped sweep if the device test fired), whether it
 * fired, and the latest known change (at the stopped sweep, else of the
 * sweep before the last; +inf if none yet).  STC_EDEGENERATE if a sweep
 * produced no positive mass. */
stc_status stc_query(stc_handle *h, int64_t *sweeps, int32_t *stopped, double *diff_1);

/* Copy the handle's current (or stopped) iterate, normalised, to pi. */
stc_status stc_store(stc_handle *h, double *pi, int32_t where);

/* Precision switch of the mixed schedule: continue the handle's iteration in
 * FP64 from its current FP32 iterate k (the stopped sweep if the device test
 * fired).  The iterate is widened exactly, so the next FP64 sweep continues
 * the same recurrence.  The changes of sweeps k - 1 and k keep their FP32
 * values; the FP64 stopping test starts with the change of sweep k + 1, so a
 * stop after the switch always comes after at least one FP64 sweep.
 * STC_EINVAL if the handle does not sweep in FP32. */
stc_status stc_promote(stc_handle *h);

/* ---- many chains ------------------------------------------------------
 * A batch sweeps many independent chains (one handle each, of any L and m)
 * with one persistent launch per half-sweep, precision stage and padded
 * block size present: a work list of (chain, group of levels) items strided
 * over a fixed grid.  Each chain's sweep is reduced and recorded (scale,
 * change, device stopping test) by one workgroup of the next sweep's phase-A
 * launch, and the last sweep of each stc_batch_sweeps call by a finalize
 * launch.  Each (precision
 * stage, block size) present runs all the sweeps of a stc_batch_sweeps call
 * (both phases and its chains' finalize, sweep after sweep) on a side stream
 * of the batch, forked from its stream once and joined back once, so the
 * launches of different sizes overlap and need not wait for each other
 * between sweeps.  Each chain keeps its own
 * sweep number, scale ring and device stopping test, so chains admitted at
 * different times advance independently and a stopped chain stays put.  The
 * chain table and work lists live at fixed device addresses, so the
 * hipGraph that stc_batch_sweeps captures stays valid when stc_batch_set
 * changes the membership (it is captured again when the set of precision
 * stages or block sizes present changes, or nsweeps does; the call then
 * waits for the stream to drain before it releases the old graph).  Per-chain results equal those of the same chain
 * swept alone with launch variant 0 (same per-level arithmetic, same
 * fixed-order reductions). */
typedef struct stc_batch stc_batch;

/* Device bytes of a batch's tables. */
size_t stc_batch_footprint(int32_t max_chains, int64_t max_items);

/* Create a batch whose tables live in arena (caller-owned, 256-byte
 * aligned, >= stc_batch_footprint).  All its chains must have block
 * bandwidth b.  max_items bounds the work items of one half-sweep over all
 * chains: one per 1, 2 or 4 groups of levels (the tuned groups per item),
 * plus one reduction item per chain in phase A; stc_batch_set fails with
 * STC_EINVAL beyond it.  stream: the hipStream_t the batch launches on; NULL makes the
 * batch create (and later destroy) a non-blocking stream of its own, since a
 * graph cannot be captured on the null stream.  Work enqueued by
 * stc_batch_sweeps is ordered only on that stream: call stc_batch_sync
 * before reading a chain through its handle. */
stc_status stc_batch_create(int32_t max_chains, int64_t max_items, int32_t b, void *stream,
                            void *arena, size_t arena_bytes, stc_batch **out);

/* Set the batch's chains (their current iterates and precision stages) and
 * the change tolerance of the device stopping test: chains sweeping in FP32
 * under STC_MIXED stop at their switch_tol, all others at tol.  nontemporal
 * selects non-temporal block loads for the block sizes the batch has not
 * tuned (stc_batch_autotune).  Each chain takes the batch's launch variant for
 * its block size in both stages (its handle's stc_get_variant reports it), so
 * the chain swept alone does the same per-level arithmetic.  Synchronous.
 * On failure (STC_EINVAL: a bad handle, too many chains or work items) the
 * batch is left with no chains. */
stc_status stc_batch_set(stc_batch *bt, stc_handle *const *hs, int32_t count, double tol,
                         int32_t nontemporal);

/* Enqueue nsweeps sweeps of every chain of the batch on its stream, as a
 * replay of a captured hipGraph (use_graph != 0; captured on first use and
 * again when nsweeps or the set of precision stages or block sizes changes)
 * or as plain launches.  Asynchronous: use stc_batch_sync / stc_query
 * afterwards.  Known problem: a capture made right after the previous graph
 * is released has ended the process with a segmentation fault inside this
 * call (bursts of changing length back to back; a served stream whose block
 * sizes change every round), cause not yet found.  Callers that change
 * nsweeps or the batch's sizes often should pass use_graph = 0. */
stc_status stc_batch_sweeps(stc_batch *bt, int64_t nsweeps, int32_t use_graph);

/* Autotuner of the batched launch (project-written; the tile and wave shapes
 * of the many-chain launch).  For each (precision stage, padded block size)
 * present among the chains set, one at a time, it times trial_sweeps sweeps
 * of the whole batch (after 2 warm-up sweeps, stopping tests off) for every
 * launch shape: the tile of launch variants 0 to 3 (row groups per level, so
 * levels per workgroup, and plain or non-temporal block loads), 1, 2 or 4
 * groups of levels per work item, and a persistent grid of 2, 4, 8 or 16
 * workgroups per compute unit; it keeps the fastest.  The tuned shapes stay
 * with the batch (the next stc_batch_sweeps captures its graph again) and
 * apply to chains set later.  It moves the chains' iterates: each is left
 * loaded with e/N in the first stage of its precision schedule, with the
 * batch's variants.  ms_per_sweep (may be NULL): the batch's sweep time with
 * the kept shapes.  STC_EINVAL if no chains are set. */
stc_status stc_batch_autotune(stc_batch *bt, int32_t trial_sweeps, double *ms_per_sweep);

/* The batch's launch shape for stage (STC_FP64 or STC_FP32) and padded block
 * size mp (8, 16, 32, 64 or 128): the launch variant (bits 0 and 1), the
 * groups of levels per work item and the workgroups of the persistent grid.
 * Any pointer may be NULL. */
stc_status stc_batch_get_tile(const stc_batch *bt, int32_t stage, int32_t mp, int32_t *variant,
                              int32_t *groups_per_item, int32_t *grid);

/* The stopping state of every chain of the batch in one device-to-host copy,
 * after the work enqueued on the batch's stream (synchronises that stream).
 * Arrays (host, may be NULL) have one entry per chain, in the order of the
 * last stc_batch_set.  Per chain the values equal what stc_query returns for
 * its handle: sweeps = the sweep of the current iterate, stopped = the device
 * stopping test has fired (section 3's test on the change), diff_1 = the
 * latest change known for certain (+inf before the first), and status =
 * STC_OK or STC_EDEGENERATE (a sweep gave e^T z <= 0).  The call itself
 * returns STC_OK unless the device fails. */
stc_status stc_batch_query(stc_batch *bt, int64_t *sweeps, int32_t *stopped, double *diff_1,
                           int32_t *status);
stc_status stc_batch_sync(stc_batch *bt);
void stc_batch_destroy(stc_batch *bt);

/* Release the handle (the arena stays with the caller). */
void stc_destroy(stc_handle *h);

const char *stc_status_string(stc_status s);
const char *stc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STC_H */
