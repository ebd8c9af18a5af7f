// Host runtime of the staircase solver: validation and packing of the block
// generator, arena layout, the solve loop with its stopping tests, and the
// C ABI declared in include/stc.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <sched.h>

#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "../../include/stc.h"
#include "stc_internal.h"

using namespace stc;

namespace {

thread_local char g_err[512] = "";

stc_status fail(stc_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(STC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Host threads for validation and packing: the CPUs this process may run on,
// at most 16, and one for inputs too small to pay for starting threads.
int host_threads(double bytes) {
    if (bytes < 8.0 * (1 << 20)) return 1;
    cpu_set_t set;
    int n = 1;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) n = CPU_COUNT(&set);
    return std::max(1, std::min(n, 16));
}

// Run f(k, i0, i1) over contiguous sub-ranges k = 0.. of the levels
// [l0, l1) on up to `threads` host threads (the caller's thread takes range
// 0).  Returns the number of ranges.
template <typename F>
int for_level_ranges(int l0, int l1, int threads, F f) {
    const int n = l1 - l0;
    const int t = std::max(1, std::min(threads, n));
    if (t == 1) {
        f(0, l0, l1);
        return 1;
    }
    std::vector<std::thread> pool;
    pool.reserve(t - 1);
    for (int k = 1; k < t; ++k) {
        const int a = l0 + (int)((long long)n * k / t), e = l0 + (int)((long long)n * (k + 1) / t);
        pool.emplace_back([=, &f]() { f(k, a, e); });
    }
    f(0, l0, l0 + (int)((long long)n / t));
    for (auto &th : pool) th.join();
    return t;
}

// First error found by any packing thread, by lowest level.
struct LevelError {
    int level = -1;
    std::string msg;
};

// Sub-allocation plan of one chain inside its arena.
struct Layout {
    int MP = 0, NB = 0;
    bool fp32 = false;          // FP32 copies of blocks and iterates
    bool sparse = false;        // off-diagonal blocks swept from ELL storage
    bool general = false;       // any block pattern: one near / far ELL per level
    size_t ell_tab = 0, ell_v64 = 0, ell_v32 = 0, ell_idx = 0;
    long long ell_slots = 0;    // sum over blocks of 4 x quads (value slots)
    size_t ell_meta = 0;        // bytes of the blocks' q_j and round offsets
    size_t gen_tab = 0, gen_v64 = 0, gen_v32 = 0, gen_idx = 0;
    long long gen_slots = 0;    // sum over levels of (Kn + Kf) * MP
    // Krylov workspace: r + 3 FP64 vectors (x, w, v_0 .. v_r), the apply
    // state, scratch partials of its sweeps, dot partials, small scalars
    int kr = 0;
    size_t kvec = 0, kst = 0, kpart = 0, kdot = 0, kh = 0;
    size_t blk64 = 0, diag64 = 0, blk32 = 0, w64 = 0, w32 = 0, wres = 0, io = 0;
    size_t part_sum = 0, part_diff = 0, part_aux = 0, off = 0, sizes = 0, state = 0, flow = 0;
    size_t rbuf = 0;            // large blocks: r_i of the gather launches (L x MP elements)
    size_t inv_scr = 0;         // large blocks: the inverse's panel scratch
    size_t zpart = 0;           // large blocks, STC_JGS: row parts of a split apply
    size_t nparts = 0, naux = 0;
    size_t total = 0;
};

int level_size(const stc_generator *g, int i) { return g->sizes ? g->sizes[i] : g->m; }

// Nonzeros of each column of the gather-oriented block Q_{k,i}, k = i + d
// (cnt[0..m), zero beyond the level's size; nothing for d = 0 or an absent
// neighbour).  Returns false if there is no such block.
bool ell_column_counts(const stc_generator *g, int i, int d, int *cnt) {
    const int k = i + d, b = g->b, m = g->m, NB = 2 * b + 1;
    std::fill(cnt, cnt + m, 0);
    if (k < 0 || k >= g->L || d == 0) return false;
    const double *Q = g->blocks + ((size_t)k * NB + (-d + b)) * (size_t)m * m;
    const int nk = level_size(g, k), ni = level_size(g, i);
    for (int j = 0; j < ni; ++j)
        for (int r = 0; r < nk; ++r) cnt[j] += Q[(size_t)r * m + j] != 0.0;
    return true;
}

// Storage shape of one sparse off-diagonal block (see EllEntry): Kq rounds,
// quads = sum of q_j over the columns.
struct EllShape {
    int Kq = 0;
    long long quads = 0;
};

EllShape ell_shape_of(const int *cnt, int m) {
    EllShape e;
    for (int j = 0; j < m; ++j) {
        const int qj = (cnt[j] + 3) / 4;
        e.Kq = std::max(e.Kq, qj);
        e.quads += qj;
    }
    return e;
}

// Bytes of a block's q_j and round offsets, rounded up to 4.
size_t ell_meta_bytes(int MP, int Kq) { return ((size_t)MP + 2 * ((size_t)Kq + 1) + 3) / 4 * 4; }

bool csr_input(const stc_generator *g) { return !g->blocks && g->csr_rowptr; }

// State offsets of the levels (prefix sums of the sizes), and the level of
// every state.
void level_offsets(const stc_generator *g, std::vector<long long> *off, std::vector<int> *lev) {
    off->assign(g->L + 1, 0);
    for (int i = 0; i < g->L; ++i) (*off)[i + 1] = (*off)[i] + level_size(g, i);
    if (lev) {
        lev->resize((*off)[g->L]);
        for (int i = 0; i < g->L; ++i)
            std::fill(lev->begin() + (*off)[i], lev->begin() + (*off)[i + 1], i);
    }
}

// EllShape of every block [L][2b+1] (empty for the diagonal and absent
// blocks).  For CSR input the nonzeros of each column of each
// gather-oriented block Q_{i+d,i} are counted from the entries directly;
// entries outside the band or the matrix are skipped here (setup rejects
// them).  Returns false if the CSR row pointers are malformed.
bool ell_shape_table(const stc_generator *g, std::vector<EllShape> *shapes) {
    const int L = g->L, b = g->b, m = g->m, NB = 2 * b + 1;
    shapes->assign((size_t)L * NB, EllShape());
    if (!csr_input(g)) {
        std::vector<int> cnt(m);
        for (int i = 0; i < L; ++i)
            for (int d = -b; d <= b; ++d)
                if (ell_column_counts(g, i, d, cnt.data()))
                    (*shapes)[(size_t)i * NB + d + b] = ell_shape_of(cnt.data(), m);
        return true;
    }
    std::vector<long long> off;
    std::vector<int> lev;
    level_offsets(g, &off, &lev);
    const long long N = off[L];
    const int64_t *rp = g->csr_rowptr;
    if (rp[0] != 0) return false;
    std::vector<int> cnt((size_t)L * NB * m, 0);
    for (long long r = 0; r < N; ++r) {
        if (rp[r + 1] < rp[r]) return false;
        const int k = lev[r];
        for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
            const long long c = g->csr_col[p];
            if (c < 0 || c >= N || g->csr_val[p] == 0.0) continue;
            const int i = lev[c], d = k - i;
            if (d == 0 || d < -b || d > b) continue;
            ++cnt[((size_t)i * NB + d + b) * m + (c - off[i])];
        }
    }
    for (size_t blk = 0; blk < (size_t)L * NB; ++blk)
        (*shapes)[blk] = ell_shape_of(cnt.data() + blk * m, m);
    return true;
}

// Near and far ELL widths of every level of a generator of any block pattern
// (CSR input): per column c of level i, the nonzero off-diagonal entries
// Q_{r,c} with r in level i - 1 or i + 1 (near) or in any other level except
// i (far); the widths are the longest column of each kind, rounded up to a
// multiple of 4.  Entries of level i itself go to the dense diagonal block.
// Entries outside the matrix are skipped here (setup rejects them).  Returns
// false if the row pointers are malformed.
bool gen_K_table(const stc_generator *g, std::vector<int> *Kn, std::vector<int> *Kf) {
    const int L = g->L;
    std::vector<long long> off;
    std::vector<int> lev;
    level_offsets(g, &off, &lev);
    const long long N = off[L];
    const int64_t *rp = g->csr_rowptr;
    if (rp[0] != 0) return false;
    std::vector<int> cn(N, 0), cf(N, 0);
    for (long long r = 0; r < N; ++r) {
        if (rp[r + 1] < rp[r]) return false;
        const int k = lev[r];
        for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
            const long long c = g->csr_col[p];
            if (c < 0 || c >= N || g->csr_val[p] == 0.0) continue;
            const int i = lev[c];
            if (i == k) continue;
            ++((k == i - 1 || k == i + 1) ? cn : cf)[c];
        }
    }
    Kn->assign(L, 0);
    Kf->assign(L, 0);
    for (int i = 0; i < L; ++i) {
        int a = 0, b = 0;
        for (long long c = off[i]; c < off[i + 1]; ++c) {
            a = std::max(a, cn[c]);
            b = std::max(b, cf[c]);
        }
        (*Kn)[i] = (a + 3) / 4 * 4;
        (*Kf)[i] = (b + 3) / 4 * 4;
    }
    return true;
}

// Row-block access to the generator's host input during setup.  Dense input
// is read in place.  CSR input is scattered, a range of block rows at a time
// (on the packing threads), into a zeroed staging copy of the dense layout
// [level][2b+1][m][m]; the entries are checked on the way.
struct BlockSource {
    const stc_generator *g = nullptr;
    int L = 0, m = 0, b = 0, NB = 0;
    std::vector<long long> off;
    std::vector<int> lev;
    std::vector<double> buf;
    int lo = 0, hi = 0;

    explicit BlockSource(const stc_generator *gen) : g(gen), L(gen->L), m(gen->m), b(gen->b) {
        NB = 2 * b + 1;
        if (csr_input(g)) level_offsets(g, &off, &lev);
    }
    // Q_{lev, lev + slot - b}, m x m row-major
    const double *at(int level, int slot) const {
        const size_t ms = (size_t)m * m;
        if (!csr_input(g)) return g->blocks + ((size_t)level * NB + slot) * ms;
        return buf.data() + ((size_t)(level - lo) * NB + slot) * ms;
    }
    // Make block rows [l0, l1) (clamped to the levels) readable through at().
    // CSR: on a bad entry, *err names the lowest level that has one.
    void load(int l0, int l1, int threads, LevelError *err) {
        if (!csr_input(g)) return;
        lo = std::max(0, l0);
        hi = std::min(L, l1);
        const size_t ms = (size_t)m * m;
        buf.resize((size_t)(hi - lo) * NB * ms);
        const long long N = off[L];
        std::vector<LevelError> errs(threads);
        for_level_ranges(lo, hi, threads, [&](int t, int i0, int i1) {
            std::fill(buf.begin() + (size_t)(i0 - lo) * NB * ms,
                      buf.begin() + (size_t)(i1 - lo) * NB * ms, 0.0);
            std::vector<long long> cols;
            char msg[256];
            for (int i = i0; i < i1; ++i)
                for (long long r = off[i]; r < off[i + 1]; ++r) {
                    const int64_t p0 = g->csr_rowptr[r], p1 = g->csr_rowptr[r + 1];
                    if (p1 < p0 || (r == 0 && p0 != 0)) {
                        snprintf(msg, sizeof(msg), "CSR row pointers fall at row %lld", r);
                        errs[t] = LevelError{i, msg};
                        return;
                    }
                    cols.clear();
                    for (int64_t p = p0; p < p1; ++p) {
                        const long long c = g->csr_col[p];
                        if (c < 0 || c >= N) {
                            snprintf(msg, sizeof(msg), "CSR column %lld of row %lld is outside 0..%lld",
                                     c, r, N - 1);
                            errs[t] = LevelError{i, msg};
                            return;
                        }
                        const int k = lev[c];
                        if (k < i - b || k > i + b) {
                            snprintf(msg, sizeof(msg),
                                     "CSR entry (%lld, %lld) joins levels %d and %d: outside the "
                                     "block band %d", r, c, i, k, b);
                            errs[t] = LevelError{i, msg};
                            return;
                        }
                        cols.push_back(c);
                        buf[((size_t)(i - lo) * NB + (k - i + b)) * ms +
                            (size_t)(r - off[i]) * m + (c - off[k])] = g->csr_val[p];
                    }
                    std::sort(cols.begin(), cols.end());
                    for (size_t q = 1; q < cols.size(); ++q)
                        if (cols[q] == cols[q - 1]) {
                            snprintf(msg, sizeof(msg), "CSR row %lld repeats column %lld", r, cols[q]);
                            errs[t] = LevelError{i, msg};
                            return;
                        }
                }
        });
        for (const auto &e : errs)
            if (e.level >= 0 && (err->level < 0 || e.level < err->level)) *err = e;
    }
};

// Partial slots of the residual, change and load kernels (part_aux): the
// groups of the residual and change kernels, and at least the load kernel's
// 2 x 1024.
size_t aux_slots(int L, int MP) {
    const size_t groups = MP > kMaxSmallMP ? (size_t)L * big_residual_slices(MP) : (size_t)L;
    return std::max<size_t>(2 * 1024 + 8, groups + 8);
}

bool plan(const stc_generator *g, const stc_options *o, Layout *lay, int *why) {
    *why = 0;
    if (!g || !o) return false;
    if (g->L < 2) { *why = 1; return false; }
    const bool general = g->b == STC_ANY_PATTERN;
    if (!general && (g->b < 1 || g->b > kMaxBandwidth)) { *why = 2; return false; }
    const int MP = supported_mp(g->m);
    // blocks above 128: generators of any pattern only (the banded kernels stop there)
    if (!MP || (MP > 128 && !general)) { *why = 3; return false; }
    if (o->precision < STC_FP64 || o->precision > STC_MIXED) { *why = 4; return false; }
    if (o->format != STC_DENSE && o->format != STC_SPARSE) { *why = 5; return false; }
    if (!g->blocks && !(g->csr_rowptr && g->csr_col && g->csr_val)) { *why = 6; return false; }
    if (g->sizes)
        for (int i = 0; i < g->L; ++i)
            if (g->sizes[i] < 1 || g->sizes[i] > g->m) { *why = 9; return false; }
    if (g->blocks && g->csr_rowptr) { *why = 7; return false; }
    if (general && !csr_input(g)) { *why = 10; return false; }
    if (general && o->format != STC_SPARSE) { *why = 11; return false; }
    if (general && (long long)g->L * MP >= (1ll << 31)) { *why = 12; return false; }
    if (o->krylov_restart < 0 || o->krylov_restart > kMaxRestart) { *why = 13; return false; }
    if (o->method != STC_STAIRCASE && o->method != STC_JGS) { *why = 15; return false; }
    // Algorithm 1: dense band storage, or any block pattern
    if (o->method == STC_JGS &&
        ((!general && o->format != STC_DENSE) || o->krylov_restart != 0 || o->jgs_chunks < 1 ||
         o->jgs_chunks > g->L)) { *why = 16; return false; }
    Layout l;
    l.MP = MP;
    l.NB = general ? 1 : 2 * g->b + 1;   // any pattern: only the diagonal slot is dense
    l.fp32 = o->precision != STC_FP64;
    l.sparse = o->format == STC_SPARSE;
    l.general = general;
    if (l.sparse && !general) {
        std::vector<EllShape> shapes;
        if (!ell_shape_table(g, &shapes)) { *why = 8; return false; }
        for (const EllShape &e : shapes) {
            l.ell_slots += 4 * e.quads;
            if (e.Kq > 0) l.ell_meta += ell_meta_bytes(MP, e.Kq);
        }
        // the row-index pool (slots, then the blocks' q_j and round offsets)
        // is addressed with 32-bit offsets
        if (l.ell_slots + (long long)l.ell_meta >= (1ll << 31)) { *why = 14; return false; }
    }
    if (general) {
        std::vector<int> Kn, Kf;
        if (!gen_K_table(g, &Kn, &Kf)) { *why = 8; return false; }
        for (int i = 0; i < g->L; ++i) l.gen_slots += (long long)(Kn[i] + Kf[i]) * MP;
    }
    const size_t L = (size_t)g->L, bs = (size_t)MP * MP, vec = L * MP;
    size_t at = 0;
    auto take = [&](size_t bytes) { size_t p = at; at = align_up(at + bytes); return p; };
    l.blk64 = take(L * l.NB * bs * 8);
    l.diag64 = take(L * bs * 8);
    if (l.fp32) l.blk32 = take(L * l.NB * bs * 4);
    l.w64 = take(4 * vec * 8);              // four iterates in rotation
    if (l.fp32) l.w32 = take(4 * vec * 4);
    l.wres = take(vec * 8);
    l.io = take(vec * 8);
    // partial slots of one sweep: a group of levels each, or for large blocks
    // a column slice of a level each (at most MP / 64 per level)
    l.nparts = MP > kMaxSmallMP ? L * (MP / 64) + 8 : L + 8;
    l.part_sum = take(2 * l.nparts * 8);    // two sweeps: parity of s
    l.part_diff = take(2 * l.nparts * 8);
    l.naux = aux_slots(g->L, MP);
    l.part_aux = take(l.naux * 8);
    if (MP > kMaxSmallMP) {
        l.rbuf = take(vec * 8);
        l.inv_scr = take(big_invert_scratch_bytes(MP, g->L));
        if (o->method == STC_JGS) l.zpart = take(jgs_big_split_bytes(g->L, MP));
    }
    if (l.sparse && !general) {
        l.ell_tab = take(L * l.NB * sizeof(EllEntry));
        l.ell_v64 = take((size_t)l.ell_slots * 8);
        if (l.fp32) l.ell_v32 = take((size_t)l.ell_slots * 4);
        l.ell_idx = take((size_t)l.ell_slots + l.ell_meta);
    }
    if (general) {
        l.gen_tab = take(L * sizeof(GenEntry));
        l.gen_v64 = take((size_t)l.gen_slots * 8);
        if (l.fp32) l.gen_v32 = take((size_t)l.gen_slots * 4);
        l.gen_idx = take((size_t)l.gen_slots * 4);
    }
    if (o->krylov_restart > 0) {
        l.kr = o->krylov_restart;
        l.kvec = take((size_t)(l.kr + 3) * vec * 8);
        l.kst = take(sizeof(DevState));
        l.kpart = take(2 * l.nparts * 8);
        l.kdot = take((size_t)kDotGroups * (l.kr + 2) * 8);
        // scalars, the cycle's y, and per step the norm and both Gram-Schmidt
        // passes' coefficients for a whole cycle
        l.kh = take((size_t)(2 * (size_t)l.kr * (l.kr + 2) + 2 * l.kr + 32) * 8);
    }
    l.off = take((L + 1) * 8);
    l.sizes = take(L * 4);
    l.state = take(sizeof(DevState));
    l.flow = take((L + 8) * sizeof(unsigned));   // progress flags of a persistent burst
    l.total = at;
    *lay = l;
    return true;
}

}  // namespace

struct stc_handle {
    int L = 0, m = 0, b = 0, MP = 0, NB = 0;
    int precision = STC_FP64, stair_type = 1, stop = STC_STOP_DIFF, check_every = 1;
    double switch_tol = 1e-6;
    hipStream_t stream = nullptr;
    int device = 0;
    Layout lay;
    char *base = nullptr;
    // device views
    double *blk64 = nullptr, *diag64 = nullptr, *w64 = nullptr, *wres = nullptr, *io = nullptr;
    float *blk32 = nullptr, *w32 = nullptr;
    double *part_sum = nullptr, *part_diff = nullptr, *part_aux = nullptr;
    long long *off = nullptr;
    int *sizes_d = nullptr;
    DevState *st = nullptr;
    std::vector<int> sizes;
    long long N = 0;
    int variant[2] = {0, 0};   // sweep-kernel launch variant for FP64 [0] / FP32 [1] stages
    int method = STC_STAIRCASE;
    int chunks = 0;            // STC_JGS: chunks of levels (workgroups of a sweep)
    bool sparse = false;
    EllEntry *ell_tab = nullptr;
    double *ell_v64 = nullptr;
    float *ell_v32 = nullptr;
    unsigned char *ell_idx = nullptr;
    std::vector<EllShape> ell_shape;   // [L][NB] storage shape per block
    // any block pattern
    bool general = false;
    GenEntry *gen_tab = nullptr;
    double *gen_v64 = nullptr;
    float *gen_v32 = nullptr;
    int *gen_idx = nullptr;
    void *rbuf = nullptr;             // large blocks: the gather launches' r_i
    void *zpart = nullptr;            // large blocks, STC_JGS: row parts of a split apply
    std::vector<GenEntry> gen_host;   // the table, for the byte counts
    // Krylov workspace (stc_solve_gmres)
    int kr = 0;
    bool keep_all = false;   // stc_solve_gmres keeps every cycle (no safeguard)
    double *kX = nullptr, *kW = nullptr, *kV = nullptr, *kpart = nullptr, *kdot = nullptr,
           *kh = nullptr;
    DevState *kst = nullptr;
    double gen_vin[2] = {0.0, 0.0};   // distinct source values read by phase A / B
    unsigned *flow_flags = nullptr;   // progress flags of a persistent burst
    int flow_res[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}};   // resident blocks, cached
    long long wall_hz = 100000000;    // device wall clock rate
    // iteration state
    long long s = 0;        // sweeps done since the last load
    bool stage32 = false;   // current iterate lives in the FP32 rotation
    long long iters32 = 0;  // sweeps done in FP32 since the last load
};

namespace {

void *wbuf(stc_handle *h, bool fp32, long long s) {
    const size_t vec = (size_t)h->L * h->MP;
    const int k = (int)(((s % 4) + 4) % 4);
    if (fp32) return h->w32 + k * vec;
    return h->w64 + k * vec;
}

int sweep_slots(stc_handle *h) {
    const bool f32 = h->stage32;
    if (h->method == STC_JGS)   // per chunk; per (level, slice) on the large blocks
        return h->MP > kMaxSmallMP ? h->L * big_slices(f32 ? 4 : 8, h->MP) : h->chunks;
    const int vv = h->sparse ? kEllGeometry : h->variant[f32 ? 1 : 0];
    const int bytes = f32 ? 4 : 8;
    const int pA = (h->stair_type == 1) ? 0 : 1;
    return phase_groups(bytes, h->MP, h->L, pA, vv) + phase_groups(bytes, h->MP, h->L, 1 - pA, vv);
}

bool folds(stc_handle *h) { return sweep_slots(h) <= kFoldSlots; }

// Enqueue sweep s: phase A, phase B and, for chains with more partial slots
// than the reduction workgroup of phase B takes, a finalize launch.  first:
// the first sweep of a burst (the previous sweep was recorded by a flush, a
// load or a batch, so phase B does not reduce it again).  With ev != nullptr
// an event is recorded after phase A (ev[0]), after phase B (ev[1]) and after
// a finalize launch (ev[2], only when one is enqueued).
// Events of one profiled sweep: each phase's dispatch, and the per-sweep
// finalize launch of long chains.
struct SweepTimers {
    LaunchTimer a, b;
    hipEvent_t fin0 = nullptr, fin1 = nullptr;
};

// One sweep of Algorithm 1 (STC_JGS): a single launch (on the large blocks,
// a gather and an apply launch per level of a chunk) whose extra workgroup
// records sweep s - 1, then a finalize launch if the partials are too many
// to fold.
hipError_t enqueue_sweep_jgs(stc_handle *h, long long s, double tol, const SweepTimers *tm,
                             bool first) {
    const bool f32 = h->stage32;
    SweepLaunch a;
    a.blk = f32 ? (const void *)h->blk32 : (const void *)h->blk64;
    a.w_old = wbuf(h, f32, s - 1);
    a.w_d1 = wbuf(h, f32, s - 2);
    a.w_d2 = wbuf(h, f32, s - 3);
    a.w_new = wbuf(h, f32, s);
    a.part_sum = h->part_sum + (s & 1) * h->lay.nparts;
    a.part_diff = h->part_diff + (s & 1) * h->lay.nparts;
    a.st = h->st;
    a.L = h->L;
    a.s = s;
    a.tol = tol;
    a.parity = 0;
    a.slot0 = 0;
    const int nslots = sweep_slots(h);
    a.nslots = nslots;
    const bool fold_ok = nslots <= kFoldSlots;
    a.fold = (fold_ok && !first && s >= 2) ? 1 : 0;
    a.prev_nslots = nslots;
    a.prev_sum = h->part_sum + ((s - 1) & 1) * h->lay.nparts;
    a.prev_diff = h->part_diff + ((s - 1) & 1) * h->lay.nparts;
    const bool nt = variant_nt(h->variant[f32 ? 1 : 0]);
    const void *gval = f32 ? (const void *)h->gen_v32 : (const void *)h->gen_v64;
    const LaunchTimer t = tm ? tm->a : LaunchTimer();
    hipError_t e;
    if (h->general && h->MP > kMaxSmallMP)
        e = launch_sweep_jgs_big(f32 ? 4 : 8, h->MP, nt, h->chunks, a, h->gen_tab, gval,
                                 h->gen_idx, h->rbuf, h->zpart, h->stream, t);
    else if (h->general)
        e = launch_sweep_jgs_gen(f32 ? 4 : 8, h->MP, nt, h->chunks, a, h->gen_tab, gval,
                                 h->gen_idx, h->stream, t);
    else
        e = launch_sweep_jgs(f32 ? 4 : 8, h->MP, h->b, nt, h->chunks, a, h->stream, t);
    if (!fold_ok) {
        if (e == hipSuccess && tm) e = hipEventRecord(tm->fin0, h->stream);
        if (e == hipSuccess)
            e = launch_finalize_sweep(a.part_sum, a.part_diff, nslots, h->st, s, tol, h->stream);
        if (e == hipSuccess && tm) e = hipEventRecord(tm->fin1, h->stream);
    }
    return e;
}

hipError_t enqueue_sweep(stc_handle *h, long long s, double tol, const SweepTimers *tm,
                         bool first) {
    if (h->method == STC_JGS) return enqueue_sweep_jgs(h, s, tol, tm, first);
    const bool f32 = h->stage32;
    const int v = h->variant[f32 ? 1 : 0];
    SweepLaunch a;
    a.blk = f32 ? (const void *)h->blk32 : (const void *)h->blk64;
    a.w_old = wbuf(h, f32, s - 1);
    a.w_d1 = wbuf(h, f32, s - 2);
    a.w_d2 = wbuf(h, f32, s - 3);
    a.w_new = wbuf(h, f32, s);
    a.part_sum = h->part_sum + (s & 1) * h->lay.nparts;
    a.part_diff = h->part_diff + (s & 1) * h->lay.nparts;
    a.st = h->st;
    a.L = h->L;
    a.s = s;
    a.tol = tol;
    const int pA = (h->stair_type == 1) ? 0 : 1;
    const int pB = 1 - pA;
    const int bytes = f32 ? 4 : 8;
    const int vv = h->sparse ? kEllGeometry : v;   // the sparse kernel's fixed tile
    const int gA = phase_groups(bytes, h->MP, h->L, pA, vv);
    const int gB = phase_groups(bytes, h->MP, h->L, pB, vv);
    const bool fold_ok = gA + gB <= kFoldSlots;
    a.nslots = gA + gB;
    a.fold = 0;
    a.prev_nslots = gA + gB;
    a.prev_sum = h->part_sum + ((s - 1) & 1) * h->lay.nparts;
    a.prev_diff = h->part_diff + ((s - 1) & 1) * h->lay.nparts;
    a.parity = pA;
    a.slot0 = 0;
    const void *ev_val = f32 ? (const void *)h->ell_v32 : (const void *)h->ell_v64;
    auto phase = [&](bool phb) {
        const LaunchTimer t = tm ? (phb ? tm->b : tm->a) : LaunchTimer();
        if (h->general)
            return launch_sweep_phase_gen(bytes, h->MP, phb, (v & 2) != 0, a, h->gen_tab,
                                          f32 ? (const void *)h->gen_v32 : (const void *)h->gen_v64,
                                          h->gen_idx, h->rbuf, h->stream, t);
        if (h->sparse)
            return launch_sweep_phase_ell(bytes, h->MP, h->b, phb, a, h->ell_tab, ev_val,
                                          h->ell_idx, h->stream, t);
        return launch_sweep_phase(bytes, h->MP, h->b, phb, v, a, h->stream, t);
    };
    hipError_t e = phase(false);
    a.parity = pB;
    a.slot0 = gA;
    // phase B's extra workgroup records sweep s-1 (unless a flush or a batch
    // already did, i.e. at the start of a burst)
    a.fold = (fold_ok && !first && s >= 2) ? 1 : 0;
    if (e == hipSuccess) e = phase(true);
    if (!fold_ok) {
        if (e == hipSuccess && tm) e = hipEventRecord(tm->fin0, h->stream);
        if (e == hipSuccess)
            e = launch_finalize_sweep(a.part_sum, a.part_diff, gA + gB, h->st, s, tol, h->stream);
        if (e == hipSuccess && tm) e = hipEventRecord(tm->fin1, h->stream);
    }
    return e;
}

// Finish a burst that ended with sweep n: record sweep n (the reduction the
// next sweep's phase B would have done) and the changes of sweeps n-1 and n,
// which the lagged partials have not measured yet, with the device stopping
// test in sweep order.  After it the state is complete up to sweep n.
hipError_t end_burst(stc_handle *h, long long n, double tol, bool recorded = false) {
    if (n < 1) return hipSuccess;
    hipError_t e = hipSuccess;
    if (folds(h) && !recorded)
        e = launch_finalize_sweep(h->part_sum + (n & 1) * h->lay.nparts,
                                  h->part_diff + (n & 1) * h->lay.nparts, sweep_slots(h), h->st,
                                  n, tol, h->stream);
    const bool f32 = h->stage32;
    const int vv = h->sparse ? kEllGeometry : h->variant[f32 ? 1 : 0];
    const int pA = (h->stair_type == 1) ? 0 : 1;
    for (long long k = n - 1; k <= n && e == hipSuccess; ++k) {
        if (k < 1) continue;
        if (h->method == STC_JGS)
            e = launch_diff_jgs(f32 ? 4 : 8, h->MP, wbuf(h, f32, k), wbuf(h, f32, k - 1), h->L,
                                h->chunks, h->st, k, h->part_aux, h->stream, tol);
        else
            e = launch_diff(f32 ? 4 : 8, h->MP, vv, wbuf(h, f32, k), wbuf(h, f32, k - 1), h->L,
                            pA, h->st, k, h->part_aux, h->stream, tol);
    }
    return e;
}

// Streaming blocks of a persistent burst for the handle's current stage: one
// block per group at most, every block owning at least one group of each
// phase, all of them and the folder resident at once; 0 when the stage has
// no persistent form.
int flow_blocks(stc_handle *h) {
    const bool f32 = h->stage32;
    const int v = h->variant[f32 ? 1 : 0];
    if (h->sparse || h->method == STC_JGS || !variant_flow(v)) return 0;
    int &res = h->flow_res[f32 ? 1 : 0][v & 3];
    if (res < 0) res = flow_resident_blocks(f32 ? 4 : 8, h->MP, h->b, v);
    const int bytes = f32 ? 4 : 8;
    const int pA = (h->stair_type == 1) ? 0 : 1;
    const int gA = phase_groups(bytes, h->MP, h->L, pA, v);
    const int gB = phase_groups(bytes, h->MP, h->L, 1 - pA, v);
    // as many blocks as fit, with the groups spread evenly (k or k-1 each)
    const int n = std::min(gA, gB);
    if (res < 2) return 0;
    const int k = (n + res - 2) / (res - 1);
    const int G = (n + k - 1) / k;
    return G >= 1 ? G : 0;
}

// Sweeps s0+1 .. s0+n as one persistent launch (it records them all).
hipError_t enqueue_flow(stc_handle *h, long long s0, long long n, double tol) {
    const bool f32 = h->stage32;
    const int v = h->variant[f32 ? 1 : 0];
    const int bytes = f32 ? 4 : 8;
    const int pA = (h->stair_type == 1) ? 0 : 1;
    FlowLaunch f;
    f.blk = f32 ? (const void *)h->blk32 : (const void *)h->blk64;
    for (int k = 0; k < 4; ++k) f.w[k] = wbuf(h, f32, k);
    f.part_sum = h->part_sum;
    f.part_diff = h->part_diff;
    f.nparts = (int)h->lay.nparts;
    f.st = h->st;
    f.L = h->L;
    f.parity_a = pA;
    f.groups_a = phase_groups(bytes, h->MP, h->L, pA, v);
    f.groups_b = phase_groups(bytes, h->MP, h->L, 1 - pA, v);
    f.G = flow_blocks(h);
    f.flags = h->flow_flags;
    f.s0 = s0;
    f.n = (int)n;
    f.tol = tol;
    f.timeout_ticks = 2 * h->wall_hz;   // no legitimate wait comes near two seconds
    return launch_sweep_flow(bytes, h->MP, h->b, v, f, h->stream);
}

// Enqueue sweeps s0+1 .. s0+n as one burst, state recorded at the end.
stc_status run_burst(stc_handle *h, long long s0, long long n, double tol) {
    if (n >= 1 && n <= (1ll << 30) && flow_blocks(h) > 0) {
        HIP_TRY(enqueue_flow(h, s0, n, tol));
        HIP_TRY(end_burst(h, s0 + n, tol, true));
        return STC_OK;
    }
    for (long long j = 1; j <= n; ++j) HIP_TRY(enqueue_sweep(h, s0 + j, tol, nullptr, j == 1));
    HIP_TRY(end_burst(h, s0 + n, tol));
    return STC_OK;
}

// Default launch variant before any tuning: non-temporal block streams once
// the blocks of a stage exceed the 256 MB last-level cache, four row groups
// per level for blocks of 64 and more.
int default_variant(int MP, double block_bytes) {
    int v = 0;
    if (MP >= 64) v |= 1;
    if (block_bytes > 256.0 * (1 << 20)) v |= 2;
    return v;
}

struct HostState {
    int stop_flag, status;
    long long stop_sweep, last_sweep;
    double residual, x_sum;
    int bad_blocks;
};

stc_status read_state(stc_handle *h, HostState *hs) {
    DevState tmp;
    // only the scalar tail is needed; copy from residual onwards
    const size_t off = offsetof(DevState, residual);
    HIP_TRY(hipMemcpyAsync(reinterpret_cast<char *>(&tmp) + off,
                           reinterpret_cast<char *>(h->st) + off, sizeof(DevState) - off,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (tmp.status == kDevTimeout)
        return fail(STC_EDEVICE, "a persistent sweep launch gave up waiting for another block");
    hs->stop_flag = tmp.stop_flag;
    hs->status = tmp.status;
    hs->stop_sweep = tmp.stop_sweep;
    hs->last_sweep = tmp.last_sweep;
    hs->residual = tmp.residual;
    hs->x_sum = tmp.x_sum;
    hs->bad_blocks = tmp.bad_blocks;
    return STC_OK;
}

stc_status read_ring(stc_handle *h, const double *ring_dev, long long s, double *out) {
    HIP_TRY(hipMemcpyAsync(out, ring_dev + (s & kRingMask), sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return STC_OK;
}

// Load x (compact, N; NULL = e/N) as W_0 of the given precision stage and
// reset the sweep counter.
stc_status load_vector_stage(stc_handle *h, const double *x, int32_t where, bool fp32) {
    const double *src = x;
    if (x && where == STC_MEM_HOST) {
        HIP_TRY(hipMemcpyAsync(h->io, x, sizeof(double) * h->N, hipMemcpyHostToDevice, h->stream));
        src = h->io;
    } else if (!x) {
        std::vector<double> e(h->N, 1.0 / (double)h->N);
        HIP_TRY(hipMemcpyAsync(h->io, e.data(), sizeof(double) * h->N, hipMemcpyHostToDevice,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        src = h->io;
    }
    h->stage32 = fp32;
    h->s = 0;
    h->iters32 = 0;
    HIP_TRY(launch_reset_state(h->st, h->stream));
    HIP_TRY(launch_load(h->stage32 ? 4 : 8, h->MP, src, h->off, h->sizes_d, h->L,
                        wbuf(h, h->stage32, 0), h->part_aux, (int)h->lay.naux, h->st, 0,
                        h->stream));
    HostState hs;
    stc_status rc = read_state(h, &hs);
    if (rc != STC_OK) return rc;
    if (hs.status == kDevBadStart)
        return fail(STC_EINVAL, "start vector must be >= 0, finite, with a positive sum "
                                "(sum = %g)", hs.x_sum);
    return STC_OK;
}

// Load into the first stage of the handle's precision schedule.
stc_status load_vector(stc_handle *h, const double *x, int32_t where) {
    return load_vector_stage(h, x, where, h->precision != STC_FP64);
}

// ||Q^T x||_1 of the padded iterate w (scaled by inv_sigma[slot]; slot < 0:
// as given) into DevState::residual, or into *out (device) when out is set.
// The per-group partials go to part (the handle's own by default).
hipError_t enqueue_residual(stc_handle *h, bool f32, const void *w, long long slot,
                            double *part = nullptr, double *out = nullptr) {
    if (!part) part = h->part_aux;
    if (h->general)
        return launch_residual_gen(f32 ? 4 : 8, h->MP, h->diag64, h->gen_tab, h->gen_v64,
                                   h->gen_idx, w, h->L, h->st, slot, part, h->stream, out);
    return launch_residual(f32 ? 4 : 8, h->MP, h->b, h->blk64, h->diag64, w, h->L, h->st, slot,
                           part, h->stream, out);
}

// T v = M^{-1} N v (the stair splitting's iteration operator, without
// normalisation): phase A then phase B of the sweep kernels on the Krylov
// apply-state, whose scales are all 1, from v into out.  v and out are FP64,
// padded [L][MP] with zero padding; the sweeps' partial sums go to scratch.
// f32: the sweeps run on the FP32 blocks, from v rounded to FP32 (in the
// first FP32 iterate buffer) into the second, widened exactly into out.
hipError_t enqueue_apply(stc_handle *h, const double *v, double *out, bool f32 = false) {
    const int bytes = f32 ? 4 : 8;
    const int var = h->variant[f32 ? 1 : 0] & 3;   // the per-phase form of the stage's variant
    const int vv = h->sparse ? kEllGeometry : var;
    const int pA = (h->stair_type == 1) ? 0 : 1;
    const int gA = phase_groups(bytes, h->MP, h->L, pA, vv);
    const int gB = phase_groups(bytes, h->MP, h->L, 1 - pA, vv);
    const size_t n = (size_t)h->L * h->MP;
    void *src = (void *)v, *dst = out;
    if (f32) {
        src = wbuf(h, true, 0);
        dst = wbuf(h, true, 1);
        hipError_t e = launch_cast_blocks(v, (float *)src, n, h->stream);
        if (e != hipSuccess) return e;
    }
    SweepLaunch a;
    a.blk = f32 ? (const void *)h->blk32 : (const void *)h->blk64;
    a.w_old = src;
    a.w_d1 = src;
    a.w_d2 = src;
    a.w_new = dst;
    a.part_sum = h->kpart;
    a.part_diff = h->kpart + h->lay.nparts;
    a.st = h->kst;
    a.L = h->L;
    a.s = 2;   // scale slot 0 (= 1); no change term (sweep numbers >= 3 only)
    a.tol = 0.0;
    a.nslots = gA + gB;
    a.fold = 0;
    a.prev_nslots = gA + gB;
    a.prev_sum = a.part_sum;
    a.prev_diff = a.part_diff;
    hipError_t e = hipSuccess;
    for (int ph = 0; ph < 2 && e == hipSuccess; ++ph) {
        a.parity = ph == 0 ? pA : 1 - pA;
        a.slot0 = ph == 0 ? 0 : gA;
        const bool phb = ph == 1;
        if (h->general)
            e = launch_sweep_phase_gen(bytes, h->MP, phb, (var & 2) != 0, a, h->gen_tab,
                                       f32 ? (const void *)h->gen_v32 : (const void *)h->gen_v64,
                                       h->gen_idx, h->rbuf, h->stream);
        else if (h->sparse)
            e = launch_sweep_phase_ell(bytes, h->MP, h->b, phb, a, h->ell_tab,
                                       f32 ? (const void *)h->ell_v32 : (const void *)h->ell_v64,
                                       h->ell_idx, h->stream);
        else
            e = launch_sweep_phase(bytes, h->MP, h->b, phb, var, a, h->stream);
    }
    if (e == hipSuccess && f32) e = launch_widen((const float *)dst, out, n, h->stream);
    return e;
}

stc_status residual_of(stc_handle *h, bool f32, long long s, double *out) {
    HIP_TRY(enqueue_residual(h, f32, wbuf(h, f32, s), s));
    HostState hs;
    stc_status rc = read_state(h, &hs);
    if (rc != STC_OK) return rc;
    *out = hs.residual;
    return STC_OK;
}

stc_status store_vector(stc_handle *h, bool f32, long long s, double *pi, int32_t where) {
    double *dst = (where == STC_MEM_DEVICE) ? pi : h->io;
    HIP_TRY(launch_store(f32 ? 4 : 8, h->MP, wbuf(h, f32, s), h->off, h->sizes_d, h->L, h->st, s,
                         dst, h->stream));
    if (where == STC_MEM_HOST)
        HIP_TRY(hipMemcpyAsync(pi, h->io, sizeof(double) * h->N, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return STC_OK;
}

// Switch the current iterate from the FP32 rotation to the FP64 one at sweep
// k: W_k, the next sweep's input, is widened exactly, so the recorded scales
// stay valid and the next FP64 sweep continues the same recurrence.  The
// device test fires two sweeps after the change it tests, and the sweeps
// queued behind it may already have overwritten the FP32 buffers of W_{k-1}
// and W_{k-2} with later iterates.  Those buffers are widened too, only so
// that every FP64 buffer the next two sweeps read holds finite values; the
// rearm that follows (test_after = k) keeps the changes of sweeps k - 1 and
// k, which would read them, from being recorded or tested again, so the
// first FP64 stop can come at sweep k + 1.
stc_status widen_at(stc_handle *h, long long k) {
    const size_t vec = (size_t)h->L * h->MP;
    for (long long j = k; j >= 0 && j >= k - 2; --j)
        HIP_TRY(launch_widen((const float *)wbuf(h, true, j), (double *)wbuf(h, false, j), vec,
                             h->stream));
    h->stage32 = false;
    return STC_OK;
}

// Setup of a generator of any block pattern (CSR input): check every row,
// then pack the dense diagonal blocks Q_ii, the per-level near / far ELL of
// the off-diagonal entries of A = Q^T (GenEntry), and the FP32 copy of its
// values.  Levels are packed a chunk at a time, so the host holds the
// transposed entries plus one chunk of the device layout.
stc_status pack_general(stc_handle *h, const stc_generator *g) {
    const int L = h->L, MP = h->MP;
    const size_t bs = (size_t)MP * MP;
    std::vector<long long> off;
    std::vector<int> lev;
    level_offsets(g, &off, &lev);
    const long long N = off[L];
    const int64_t *rp = g->csr_rowptr;
    const int32_t *col = g->csr_col;
    const double *val = g->csr_val;

    // every row: columns in range and not repeated, off-diagonal rates >= 0
    // and finite, the row sum 0 (or the diagonal recomputed)
    std::vector<double> dg(N);
    {
        std::vector<long long> cols;
        for (long long r = 0; r < N; ++r) {
            const int i = lev[r];
            const int64_t p0 = rp[r], p1 = rp[r + 1];
            if (p1 < p0 || (r == 0 && p0 != 0))
                return fail(STC_EINVAL, "CSR row pointers fall at row %lld", r);
            cols.clear();
            for (int64_t p = p0; p < p1; ++p) {
                const long long c = col[p];
                if (c < 0 || c >= N)
                    return fail(STC_EINVAL, "CSR column %lld of row %lld is outside 0..%lld", c, r,
                                N - 1);
                cols.push_back(c);
            }
            std::sort(cols.begin(), cols.end());
            for (size_t q = 1; q < cols.size(); ++q)
                if (cols[q] == cols[q - 1])
                    return fail(STC_EINVAL, "CSR row %lld repeats column %lld", r, cols[q]);
            double out = 0.0, given = 0.0;
            for (int64_t p = p0; p < p1; ++p) {
                const long long c = col[p];
                const double v = val[p];
                if (c == r) {
                    given = v;
                    continue;
                }
                if (!(v >= 0.0) || !std::isfinite(v))
                    return fail(STC_ENOTGEN, "Q[level %d row %lld][level %d col %lld] = %g is not a rate",
                                i, r - off[i], lev[c], c - off[lev[c]], v);
                out += v;
            }
            if (g->recompute_diagonal) {
                dg[r] = -out;
            } else {
                if (!std::isfinite(given) || fabs(given + out) > 1e-10 * std::max(out, 1e-300))
                    return fail(STC_ENOTGEN, "row %lld of level %d sums to %g, not 0 (diagonal %g)",
                                r - off[i], i, given + out, given);
                dg[r] = given;
            }
        }
    }

    // the off-diagonal nonzeros of other levels by column (gather orientation),
    // rows ascending within a column
    std::vector<long long> cptr(N + 1, 0);
    for (long long r = 0; r < N; ++r)
        for (int64_t p = rp[r]; p < rp[r + 1]; ++p)
            if (val[p] != 0.0 && lev[col[p]] != lev[r]) ++cptr[col[p] + 1];
    for (long long c = 0; c < N; ++c) cptr[c + 1] += cptr[c];
    std::vector<long long> crow(cptr[N]);
    std::vector<double> cval(cptr[N]);
    {
        std::vector<long long> cur(cptr.begin(), cptr.end() - 1);
        for (long long r = 0; r < N; ++r)
            for (int64_t p = rp[r]; p < rp[r + 1]; ++p)
                if (val[p] != 0.0 && lev[col[p]] != lev[r]) {
                    const long long e = cur[col[p]]++;
                    crow[e] = r;
                    cval[e] = val[p];
                }
    }
    auto near_of = [&](int k, int i) { return k == i - 1 || k == i + 1; };

    // ELL widths (the same counts as the footprint plan)
    std::vector<GenEntry> tab(L);
    long long at = 0;
    for (int i = 0; i < L; ++i) {
        int a = 0, b = 0;
        for (long long c = off[i]; c < off[i + 1]; ++c) {
            int n = 0, f = 0;
            for (long long e = cptr[c]; e < cptr[c + 1]; ++e) ++(near_of(lev[crow[e]], i) ? n : f);
            a = std::max(a, n);
            b = std::max(b, f);
        }
        tab[i] = GenEntry{at, (a + 3) / 4 * 4, (b + 3) / 4 * 4};
        at += (long long)(tab[i].Kn + tab[i].Kf) * MP;
    }
    if (at != h->lay.gen_slots) return fail(STC_EINVAL, "CSR input changed between the plan and setup");

    // values and indices, a range of levels at a time; padding slots read a
    // state of an adjacent level, which both phases have written
    const long long chunk_slots = 8ll << 20;
    std::vector<double> v64;
    std::vector<int> ix;
    for (int l0 = 0; l0 < L;) {
        int l1 = l0 + 1;
        while (l1 < L && tab[l1].off + (long long)(tab[l1].Kn + tab[l1].Kf) * MP - tab[l0].off <= chunk_slots)
            ++l1;
        const long long s0 = tab[l0].off;
        const long long s1 = l1 < L ? tab[l1].off : at;
        v64.assign((size_t)(s1 - s0), 0.0);
        ix.assign((size_t)(s1 - s0), 0);
        for (int i = l0; i < l1; ++i) {
            const GenEntry t = tab[i];
            const int pad = (i > 0 ? i - 1 : i + 1) * MP;
            std::fill(ix.begin() + (t.off - s0), ix.begin() + (t.off - s0) + (long long)(t.Kn + t.Kf) * MP, pad);
            for (long long c = off[i]; c < off[i + 1]; ++c) {
                const int j = (int)(c - off[i]);
                int n = 0, f = 0;
                for (long long e = cptr[c]; e < cptr[c + 1]; ++e) {
                    const long long r = crow[e];
                    const int k = lev[r];
                    size_t o = (size_t)(t.off - s0);
                    if (near_of(k, i)) {
                        o += ((size_t)(n >> 2) * MP + j) * 4 + (n & 3);
                        ++n;
                    } else {
                        o += (size_t)t.Kn * MP + ((size_t)(f >> 2) * MP + j) * 4 + (f & 3);
                        ++f;
                    }
                    v64[o] = cval[e];
                    ix[o] = (int)((long long)k * MP + (r - off[k]));
                }
            }
        }
        if (s1 > s0) {
            HIP_TRY(hipMemcpyAsync(h->gen_v64 + s0, v64.data(), sizeof(double) * (s1 - s0),
                                   hipMemcpyHostToDevice, h->stream));
            HIP_TRY(hipMemcpyAsync(h->gen_idx + s0, ix.data(), sizeof(int) * (s1 - s0),
                                   hipMemcpyHostToDevice, h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
        }
        l0 = l1;
    }
    HIP_TRY(hipMemcpyAsync(h->gen_tab, tab.data(), sizeof(GenEntry) * L, hipMemcpyHostToDevice,
                           h->stream));
    if (h->lay.fp32 && at > 0) HIP_TRY(launch_cast_blocks(h->gen_v64, h->gen_v32, (size_t)at, h->stream));

    // dense diagonal blocks Q_ii (padded, row-major), a chunk of levels at a time
    const int dchunk = std::max(1, (int)std::min<size_t>(L, (64u << 20) / (bs * 8)));
    std::vector<double> D((size_t)dchunk * bs);
    for (int l0 = 0; l0 < L; l0 += dchunk) {
        const int l1 = std::min(L, l0 + dchunk);
        std::fill(D.begin(), D.begin() + (size_t)(l1 - l0) * bs, 0.0);
        for (int i = l0; i < l1; ++i) {
            double *Di = D.data() + (size_t)(i - l0) * bs;
            for (long long r = off[i]; r < off[i + 1]; ++r) {
                for (int64_t p = rp[r]; p < rp[r + 1]; ++p)
                    if (lev[col[p]] == i && col[p] != r)
                        Di[(size_t)(r - off[i]) * MP + (col[p] - off[i])] = val[p];
                Di[(size_t)(r - off[i]) * MP + (r - off[i])] = dg[r];
            }
        }
        HIP_TRY(hipMemcpyAsync(h->diag64 + (size_t)l0 * bs, D.data(), sizeof(double) * (l1 - l0) * bs,
                               hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }

    // distinct source values each phase reads (per buffer), for the byte counts
    const int pA = (h->stair_type == 1) ? 0 : 1;
    for (int ph = 0; ph < 2; ++ph) {
        const int par = ph == 0 ? pA : 1 - pA;
        std::vector<char> seen_old(N, 0), seen_new(N, 0);
        double cnt = 0.0;
        for (int i = par; i < L; i += 2)
            for (long long c = off[i]; c < off[i + 1]; ++c)
                for (long long e = cptr[c]; e < cptr[c + 1]; ++e) {
                    const long long r = crow[e];
                    char &seen = (ph == 1 && near_of(lev[r], i)) ? seen_new[r] : seen_old[r];
                    if (!seen) {
                        seen = 1;
                        cnt += 1.0;
                    }
                }
        h->gen_vin[ph] = cnt;
    }
    h->gen_host = tab;
    // the kernel's one variant bit is the load policy (bit 1, non-temporal):
    // a stage whose inverse blocks and entries fit the 256 MB last-level cache
    // keeps them there from sweep to sweep (plain loads); larger ones stream
    for (int f = 0; f < 2; ++f) {
        const double sb = f ? 4.0 : 8.0;
        const double bytes = (double)L * bs * sb + (double)at * (sb + 4.0);
        h->variant[f] = bytes > 256.0 * (1 << 20) ? 2 : 0;
    }
    return STC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// the residual with caller-given staging (the allocation-free entry point in
// stc_noalloc.hip passes its static array)
// ---------------------------------------------------------------------------
namespace stc {

// Padded FP64 copy of x (L x MP) and the partials of the load and residual
// kernels, as the handle's own residual uses them.
size_t residual_staging_bytes(const stc_handle *h) {
    const size_t naux = aux_slots(h->L, h->MP);
    return align_up((size_t)h->L * h->MP * sizeof(double)) + naux * sizeof(double);
}

stc_status residual_into(stc_handle *h, const double *x, double *out, int device, char *staging,
                         size_t staging_bytes) {
    if (!h || !x || !out) return fail(STC_EINVAL, "null argument");
    if (device != h->device)
        return fail(STC_EINVAL, "the current device (%d) is not the handle's (%d)", device,
                    h->device);
    const size_t need = residual_staging_bytes(h);
    if (need > staging_bytes)
        return fail(STC_EINVAL, "this handle's residual stages %zu bytes (its padded vector "
                                "of %d x %d and the partial sums), above the allocation-free "
                                "limit of %zu bytes", need, h->L, h->MP, staging_bytes);
    double *w = reinterpret_cast<double *>(staging);
    double *aux = reinterpret_cast<double *>(staging + align_up((size_t)h->L * h->MP * sizeof(double)));
    const int naux = (int)((need - align_up((size_t)h->L * h->MP * sizeof(double))) / sizeof(double));
    // the same kernels and grids as stc_residual, so the same value bit for bit
    HIP_TRY(launch_load(8, h->MP, x, h->off, h->sizes_d, h->L, w, aux, naux, h->st, -1,
                        h->stream));
    HIP_TRY(enqueue_residual(h, false, w, -1, aux, out));
    return STC_OK;
}

stc_status report_error(stc_status s, const char *msg) { return fail(s, "%s", msg); }

}  // namespace stc

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *stc_status_string(stc_status s) {
    switch (s) {
        case STC_OK: return "STC_OK";
        case STC_EINVAL: return "STC_EINVAL: invalid argument";
        case STC_ENOTGEN: return "STC_ENOTGEN: input is not a generator";
        case STC_ESINGULAR: return "STC_ESINGULAR: singular diagonal block";
        case STC_EDEGENERATE: return "STC_EDEGENERATE: sweep produced no positive mass";
        case STC_EMAXIT: return "STC_EMAXIT: maxit reached before tol";
        case STC_ENOMEM: return "STC_ENOMEM: arena too small";
        case STC_EDEVICE: return "STC_EDEVICE: HIP error";
    }
    return "unknown status";
}

const char *stc_last_error(void) { return g_err; }

size_t stc_footprint_bytes(const stc_generator *gen, const stc_options *opt) {
    Layout l;
    int why;
    if (!plan(gen, opt, &l, &why)) return 0;
    return l.total;
}

}  // extern "C"

namespace {

// The checks and the layout of stc_setup, without the arena (stc_prepare
// shares them).
stc_status plan_setup(const stc_generator *g, const stc_options *o, Layout *lay) {
    if (g->sizes && g->L >= 2 && g->m >= 1)
        for (int i = 0; i < g->L; ++i)
            if (g->sizes[i] < 1 || g->sizes[i] > g->m)
                return fail(STC_EINVAL, "sizes[%d] = %d outside 1..%d", i, g->sizes[i], g->m);
    int why = 0;
    if (!plan(g, o, lay, &why)) {
        static const char *msg[] = {"bad arguments", "L must be >= 2",
                                    "b must be in 1..4 or STC_ANY_PATTERN",
                                    "m must be in 1..128 (1..2048 for STC_ANY_PATTERN)",
                                    "unknown precision", "unknown format",
                                    "neither blocks nor a complete CSR input given",
                                    "give blocks or CSR input, not both",
                                    "CSR row pointers must start at 0 and never fall",
                                    "a level size is outside 1..m",
                                    "a generator of any pattern (STC_ANY_PATTERN) comes as CSR input",
                                    "a generator of any pattern (STC_ANY_PATTERN) needs STC_SPARSE storage",
                                    "L * padded m must stay below 2^31",
                                    "krylov_restart must be in 0..256",
                                    "the sparse storage of the blocks exceeds 2^31 slots",
                                    "unknown method",
                                    "STC_JGS takes dense band storage or a pattern of any "
                                    "shape, no Krylov workspace and jgs_chunks in 1..L"};
        return fail(STC_EINVAL, "%s", msg[why < 17 ? why : 0]);
    }
    if (o->stair_type != 1 && o->stair_type != 2) return fail(STC_EINVAL, "stair_type must be 1 or 2");
    if (o->stop != STC_STOP_DIFF && o->stop != STC_STOP_RESIDUAL) return fail(STC_EINVAL, "bad stop rule");
    return STC_OK;
}

stc_status check_arena(const stc_options *o, const Layout &lay) {
    if (!o->arena) return fail(STC_EINVAL, "arena is NULL");
    if ((uintptr_t)o->arena % kAlign) return fail(STC_EINVAL, "arena must be 256-byte aligned");
    if (o->arena_bytes < lay.total)
        return fail(STC_ENOMEM, "arena holds %zu bytes, %zu needed", o->arena_bytes, lay.total);
    return STC_OK;
}

// A handle over the arena of o, laid out by lay, with its host fields set;
// nothing on the device yet.
stc_handle *new_handle(const stc_generator *g, const stc_options *o, const Layout &lay,
                       const std::vector<int> &sizes) {
    const int L = g->L, m = g->m, b = g->b, MP = lay.MP, NB = lay.NB;
    stc_handle *h = new stc_handle();
    h->L = L; h->m = m; h->b = b; h->MP = MP; h->NB = NB;
    h->precision = o->precision;
    h->stair_type = o->stair_type;
    h->method = o->method;
    h->chunks = o->method == STC_JGS ? o->jgs_chunks : 0;
    h->stop = o->stop;
    h->check_every = o->check_every > 0 ? o->check_every : 1;
    h->switch_tol = o->switch_tol > 0 ? o->switch_tol : 1e-6;
    h->stream = (hipStream_t)o->stream;
    h->lay = lay;
    h->base = (char *)o->arena;
    h->sizes = sizes;
    (void)hipGetDevice(&h->device);
    h->blk64 = (double *)(h->base + lay.blk64);
    h->diag64 = (double *)(h->base + lay.diag64);
    h->blk32 = lay.fp32 ? (float *)(h->base + lay.blk32) : nullptr;
    h->w64 = (double *)(h->base + lay.w64);
    h->w32 = lay.fp32 ? (float *)(h->base + lay.w32) : nullptr;
    h->wres = (double *)(h->base + lay.wres);
    h->io = (double *)(h->base + lay.io);
    h->part_sum = (double *)(h->base + lay.part_sum);
    h->part_diff = (double *)(h->base + lay.part_diff);
    h->part_aux = (double *)(h->base + lay.part_aux);
    h->off = (long long *)(h->base + lay.off);
    h->sizes_d = (int *)(h->base + lay.sizes);
    h->st = (DevState *)(h->base + lay.state);
    h->flow_flags = (unsigned *)(h->base + lay.flow);
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) == hipSuccess &&
            khz > 0)
            h->wall_hz = (long long)khz * 1000;
    }
    if (lay.kr > 0) {
        const size_t vec = (size_t)L * MP;
        h->kr = lay.kr;
        h->keep_all = o->krylov_keep_all != 0;
        h->kX = (double *)(h->base + lay.kvec);
        h->kW = h->kX + vec;
        h->kV = h->kW + vec;
        h->kst = (DevState *)(h->base + lay.kst);
        h->kpart = (double *)(h->base + lay.kpart);
        h->kdot = (double *)(h->base + lay.kdot);
        h->kh = (double *)(h->base + lay.kh);
    }
    h->sparse = lay.sparse;
    if (lay.sparse) {
        h->ell_tab = (EllEntry *)(h->base + lay.ell_tab);
        h->ell_v64 = (double *)(h->base + lay.ell_v64);
        h->ell_v32 = lay.fp32 ? (float *)(h->base + lay.ell_v32) : nullptr;
        h->ell_idx = (unsigned char *)(h->base + lay.ell_idx);
    }

    std::vector<long long> off(L + 1, 0);
    for (int i = 0; i < L; ++i) off[i + 1] = off[i] + sizes[i];
    h->N = off[L];
    {
        const double nblk = (double)L * NB * MP * MP;
        h->variant[0] = default_variant(MP, nblk * 8.0);
        h->variant[1] = default_variant(MP, nblk * 4.0);
    }

    {
        long long N = 0;
        for (int i = 0; i < L; ++i) N += sizes[i];
        h->N = N;
        const double nblk = (double)L * NB * MP * MP;
        h->variant[0] = default_variant(MP, nblk * 8.0);
        h->variant[1] = default_variant(MP, nblk * 4.0);
    }
    return h;
}

// Check block rows i0 .. i1 - 1 of a block-banded generator and pack them in
// the sweep's layout: blk holds the gather-oriented off-diagonal blocks
// (slot d + b of level i <- Q_{i+d,i}) and diag the padded Q_ii, both from
// level l0 on.  On a bad entry *err names the level and the entry.
void pack_levels(const stc_generator *g, const BlockSource &src, const std::vector<int> &sizes,
                 int MP, int l0, int i0, int i1, double *blk, double *diag, LevelError *err) {
    const int L = g->L, m = g->m, b = g->b, NB = 2 * b + 1;
    const size_t bs = (size_t)MP * MP;
    char msg[256];
    std::fill(blk + (size_t)(i0 - l0) * NB * bs, blk + (size_t)(i1 - l0) * NB * bs, 0.0);
    std::fill(diag + (size_t)(i0 - l0) * bs, diag + (size_t)(i1 - l0) * bs, 0.0);
    for (int i = i0; i < i1; ++i) {
        const int ni = sizes[i];
        // generator checks on block row i
        for (int r = 0; r < ni; ++r) {
            double out = 0.0;
            for (int d = -b; d <= b; ++d) {
                const int k = i + d;
                if (k < 0 || k >= L) continue;
                const double *row = src.at(i, d + b) + (size_t)r * m;
                for (int c = 0; c < sizes[k]; ++c) {
                    if (d == 0 && c == r) continue;
                    const double v = row[c];
                    if (!(v >= 0.0) || !isfinite(v)) {
                        snprintf(msg, sizeof(msg),
                                 "Q[level %d row %d][level %d col %d] = %g is not a rate", i, r, k,
                                 c, v);
                        *err = LevelError{i, msg};
                        return;
                    }
                    out += v;
                }
            }
            const double *qii = src.at(i, b);
            const double dg = qii[(size_t)r * m + r];
            double *D = diag + (size_t)(i - l0) * bs;
            for (int c = 0; c < ni; ++c) D[(size_t)r * MP + c] = qii[(size_t)r * m + c];
            if (g->recompute_diagonal) {
                D[(size_t)r * MP + r] = -out;
            } else if (!isfinite(dg) || fabs(dg + out) > 1e-10 * std::max(out, 1e-300)) {
                snprintf(msg, sizeof(msg), "row %d of level %d sums to %g, not 0 (diagonal %g)", r,
                         i, dg + out, dg);
                *err = LevelError{i, msg};
                return;
            }
        }
        for (int d = -b; d <= b; ++d) {
            if (d == 0) continue;
            const int k = i + d;
            if (k < 0 || k >= L) continue;
            const double *q = src.at(k, -d + b);
            double *dst = blk + ((size_t)(i - l0) * NB + (d + b)) * bs;
            for (int r = 0; r < sizes[k]; ++r)
                memcpy(dst + (size_t)r * MP, q + (size_t)r * m, sizeof(double) * sizes[i]);
        }
    }
}

// Pack levels [l0, l1) (their block rows loaded in src) on `threads` host
// threads; the first bad entry, by lowest level, as STC_ENOTGEN.
stc_status pack_range(const stc_generator *g, const BlockSource &src,
                      const std::vector<int> &sizes, int MP, int l0, int l1, int threads,
                      double *blk, double *diag) {
    std::vector<LevelError> errs(threads);
    for_level_ranges(l0, l1, threads, [&](int k, int i0, int i1) {
        pack_levels(g, src, sizes, MP, l0, i0, i1, blk, diag, &errs[k]);
    });
    const LevelError *first = nullptr;
    for (const auto &e : errs)
        if (e.level >= 0 && (!first || e.level < first->level)) first = &e;
    if (first) return fail(STC_ENOTGEN, "%s", first->msg.c_str());
    return STC_OK;
}

// The end of every setup: level offsets and sizes, the cleared state, the
// batched inverse of the diagonal blocks and the FP32 copy; then the
// singular-block check.
stc_status finish_setup(stc_handle *h, const Layout &lay, int b) {
    auto dev = [&](hipError_t e, const char *what) -> stc_status {
        if (e == hipSuccess) return STC_OK;
        return fail(STC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    };
    const int L = h->L, MP = h->MP, NB = h->NB;
    std::vector<long long> off(L + 1, 0);
    for (int i = 0; i < L; ++i) off[i + 1] = off[i] + h->sizes[i];
    stc_status rc = STC_OK;
    if ((rc = dev(hipMemcpyAsync(h->off, off.data(), sizeof(long long) * (L + 1),
                                 hipMemcpyHostToDevice, h->stream), "copy offsets")) != STC_OK)
        return rc;
    if ((rc = dev(hipMemcpyAsync(h->sizes_d, h->sizes.data(), sizeof(int) * L,
                                 hipMemcpyHostToDevice, h->stream), "copy sizes")) != STC_OK)
        return rc;
    // zero the whole state once (ring included), then the inverse
    if ((rc = dev(hipMemsetAsync(h->st, 0, sizeof(DevState), h->stream), "clear state")) != STC_OK)
        return rc;
    if ((rc = dev(launch_reset_state(h->st, h->stream), "reset")) != STC_OK) return rc;
    if (h->kr > 0 && (rc = dev(launch_kstate_init(h->kst, h->stream), "Krylov state")) != STC_OK)
        return rc;
    const hipError_t inv =
        MP > kMaxSmallMP
            ? launch_invert_big(MP, h->diag64, h->sizes_d, h->blk64, L, h->st,
                                (void *)(h->base + lay.inv_scr), h->stream)
            : launch_invert(MP, lay.general ? 0 : b, h->diag64, h->sizes_d, h->blk64, L, h->st,
                            h->stream);
    if ((rc = dev(inv, "invert")) != STC_OK) return rc;
    if (lay.fp32 &&
        (rc = dev(launch_cast_blocks(h->blk64, h->blk32, (size_t)L * NB * MP * MP, h->stream),
                  "cast")) != STC_OK)
        return rc;
    // read_state synchronises the stream: the host tables above are read
    // before they go out of scope
    HostState hs;
    if ((rc = read_state(h, &hs)) != STC_OK) return rc;
    if (hs.bad_blocks)
        return fail(STC_ESINGULAR,
                    "%d diagonal block(s) are singular: some level has states that never leave "
                    "it", hs.bad_blocks);
    return STC_OK;
}

}  // namespace

// Host half of a setup (stc_prepare): the packed blocks of a block-banded
// generator in the sweep's layout, and what the device half needs.
struct stc_prepared {
    int L = 0, m = 0, b = 0, MP = 0;
    std::vector<int> sizes;
    std::vector<double> blk, diag;
};

extern "C" {

stc_status stc_setup(const stc_generator *g, const stc_options *o, stc_handle **out) {
    if (!g || !o || !out) return fail(STC_EINVAL, "null argument");
    *out = nullptr;
    Layout lay;
    stc_status rc = plan_setup(g, o, &lay);
    if (rc != STC_OK) return rc;
    if ((rc = check_arena(o, lay)) != STC_OK) return rc;

    const int L = g->L, m = g->m, b = g->b, MP = lay.MP, NB = lay.NB;
    std::vector<int> sizes(L, m);
    if (g->sizes) std::copy(g->sizes, g->sizes + L, sizes.begin());
    stc_handle *h = new_handle(g, o, lay, sizes);
    auto cleanup = [&](stc_status s) { delete h; return s; };
    auto dev = [&](hipError_t e, const char *what) -> stc_status {
        if (e == hipSuccess) return STC_OK;
        return fail(STC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    };

    if (lay.general) {
        h->general = true;
        h->gen_tab = (GenEntry *)(h->base + lay.gen_tab);
        h->gen_v64 = (double *)(h->base + lay.gen_v64);
        h->gen_v32 = lay.fp32 ? (float *)(h->base + lay.gen_v32) : nullptr;
        h->gen_idx = (int *)(h->base + lay.gen_idx);
        h->rbuf = lay.rbuf ? (void *)(h->base + lay.rbuf) : nullptr;
        h->zpart = lay.zpart ? (void *)(h->base + lay.zpart) : nullptr;
        if ((rc = pack_general(h, g)) != STC_OK) return cleanup(rc);
    } else {
    // validate, then pack in the sweep's layout, a chunk of levels at a time;
    // the levels of a chunk are split over host threads
    const size_t bs = (size_t)MP * MP, ms = (size_t)m * m;
    const int chunk = std::max(1, (int)std::min<size_t>(L, (64u << 20) / (NB * bs * 8)));
    const int threads = host_threads((double)L * NB * ms * 8.0);
    std::vector<double> stage_blk((size_t)chunk * NB * bs), stage_diag((size_t)chunk * bs);
    BlockSource src(g);
    auto q_at = [&](int lev, int slot) { return src.at(lev, slot); };
    // block rows [l0 - b, l1 + b) are read while packing levels [l0, l1)
    auto load_rows = [&](int l0, int l1) -> stc_status {
        LevelError lerr;
        src.load(l0 - b, l1 + b, threads, &lerr);
        if (lerr.level >= 0) return fail(STC_EINVAL, "%s", lerr.msg.c_str());
        return STC_OK;
    };
    for (int l0 = 0; l0 < L; l0 += chunk) {
        const int l1 = std::min(L, l0 + chunk);
        if ((rc = load_rows(l0, l1)) != STC_OK) return cleanup(rc);
        if ((rc = pack_range(g, src, sizes, MP, l0, l1, threads, stage_blk.data(),
                             stage_diag.data())) != STC_OK)
            return cleanup(rc);
        if ((rc = dev(hipMemcpyAsync(h->blk64 + (size_t)l0 * NB * bs, stage_blk.data(),
                                     sizeof(double) * (size_t)(l1 - l0) * NB * bs,
                                     hipMemcpyHostToDevice, h->stream), "copy blocks")) != STC_OK)
            return cleanup(rc);
        if ((rc = dev(hipMemcpyAsync(h->diag64 + (size_t)l0 * bs, stage_diag.data(),
                                     sizeof(double) * (size_t)(l1 - l0) * bs,
                                     hipMemcpyHostToDevice, h->stream), "copy diagonal blocks")) != STC_OK)
            return cleanup(rc);
        if ((rc = dev(hipStreamSynchronize(h->stream), "sync")) != STC_OK) return cleanup(rc);
    }
    if (lay.sparse) {
        // every off-diagonal block by rounds of slot quads (EllEntry), levels
        // in order; the blocks' q_j and round offsets follow the slots in the
        // row-index pool
        if (!ell_shape_table(g, &h->ell_shape)) return cleanup(fail(STC_EINVAL, "bad CSR row pointers"));
        std::vector<EllEntry> tab((size_t)L * NB);
        long long at = 0;
        for (size_t q = 0; q < tab.size(); ++q) {
            tab[q] = EllEntry{at, h->ell_shape[q].Kq, 0};
            at += 4 * h->ell_shape[q].quads;
        }
        std::vector<unsigned char> meta(lay.ell_meta, 0);
        {
            size_t mo = 0;
            for (size_t q = 0; q < tab.size(); ++q) {
                if (tab[q].Kq == 0) continue;
                tab[q].meta = (int)((size_t)at + mo);
                mo += ell_meta_bytes(MP, tab[q].Kq);
            }
        }
        if ((rc = dev(hipMemcpyAsync(h->ell_tab, tab.data(), tab.size() * sizeof(EllEntry),
                                     hipMemcpyHostToDevice, h->stream), "copy ELL table")) != STC_OK)
            return cleanup(rc);
        std::vector<double> val;
        std::vector<unsigned char> idx;
        for (int l0 = 0; l0 < L; l0 += chunk) {
            const int l1 = std::min(L, l0 + chunk);
            if ((rc = load_rows(l0, l1)) != STC_OK) return cleanup(rc);
            const long long s0 = tab[(size_t)l0 * NB].off;
            const long long s1 = (l1 < L) ? tab[(size_t)l1 * NB].off : at;
            val.assign((size_t)(s1 - s0), 0.0);
            idx.assign((size_t)(s1 - s0), 0);
            // each level writes only its own blocks' slots and metadata
            for_level_ranges(l0, l1, threads, [&](int, int i0, int i1) {
                std::vector<int> cnt(MP), done(MP);
                for (int i = i0; i < i1; ++i)
                    for (int d = -b; d <= b; ++d) {
                        const EllEntry e = tab[(size_t)i * NB + d + b];
                        if (e.Kq == 0) continue;
                        const int k = i + d;
                        const double *Q = q_at(k, -d + b);    // Q_{k,i}: rows level k, cols level i
                        std::fill(cnt.begin(), cnt.end(), 0);
                        for (int j = 0; j < sizes[i]; ++j)
                            for (int r = 0; r < sizes[k]; ++r) cnt[j] += Q[(size_t)r * m + j] != 0.0;
                        // round offsets: base_t = quads of the rounds before t
                        unsigned char *qc = meta.data() + ((size_t)e.meta - (size_t)at);
                        unsigned short *base = (unsigned short *)(qc + MP);
                        base[0] = 0;
                        for (int t = 0; t < e.Kq; ++t) {
                            int n = 0;
                            for (int j = 0; j < MP; ++j) n += (cnt[j] + 3) / 4 > t;
                            base[t + 1] = (unsigned short)(base[t] + n);
                        }
                        // done[t]: columns before j with a quad in round t (rank_t)
                        std::fill(done.begin(), done.end(), 0);
                        for (int j = 0; j < MP; ++j) {
                            const int qj = (cnt[j] + 3) / 4;
                            qc[j] = (unsigned char)qj;
                            int e2 = 0;
                            for (int r = 0; r < sizes[k] && qj > 0; ++r) {
                                const double v = Q[(size_t)r * m + j];
                                if (v == 0.0) continue;
                                const int t = e2 >> 2;
                                const size_t o = (size_t)(e.off - s0) +
                                                 ((size_t)base[t] + done[t]) * 4 + (e2 & 3);
                                val[o] = v;
                                idx[o] = (unsigned char)r;
                                ++e2;
                            }
                            for (int t = 0; t < qj; ++t) ++done[t];
                        }
                    }
            });
            if (s1 > s0) {
                if ((rc = dev(hipMemcpyAsync(h->ell_v64 + s0, val.data(), sizeof(double) * (s1 - s0),
                                             hipMemcpyHostToDevice, h->stream), "copy ELL values")) != STC_OK ||
                    (rc = dev(hipMemcpyAsync(h->ell_idx + s0, idx.data(), (size_t)(s1 - s0),
                                             hipMemcpyHostToDevice, h->stream), "copy ELL rows")) != STC_OK ||
                    (rc = dev(hipStreamSynchronize(h->stream), "sync")) != STC_OK)
                    return cleanup(rc);
            }
        }
        if (!meta.empty() &&
            ((rc = dev(hipMemcpyAsync(h->ell_idx + at, meta.data(), meta.size(),
                                      hipMemcpyHostToDevice, h->stream), "copy ELL rounds")) != STC_OK ||
             (rc = dev(hipStreamSynchronize(h->stream), "sync")) != STC_OK))
            return cleanup(rc);
        if (lay.fp32 && at > 0 &&
            (rc = dev(launch_cast_blocks(h->ell_v64, h->ell_v32, (size_t)at, h->stream), "cast ELL")) != STC_OK)
            return cleanup(rc);
    }
    }
    if ((rc = finish_setup(h, lay, b)) != STC_OK) return cleanup(rc);
    *out = h;
    return STC_OK;
}

stc_status stc_prepare(const stc_generator *g, const stc_options *o, stc_prepared **out) {
    if (!g || !o || !out) return fail(STC_EINVAL, "null argument");
    *out = nullptr;
    Layout lay;
    stc_status rc = plan_setup(g, o, &lay);
    if (rc != STC_OK) return rc;
    if (lay.general || lay.sparse)
        return fail(STC_EINVAL, "stc_prepare takes dense storage of block-banded generators; "
                                "other inputs take stc_setup");
    const int L = g->L, m = g->m, b = g->b, MP = lay.MP, NB = lay.NB;
    const size_t bs = (size_t)MP * MP;
    stc_prepared *p = new (std::nothrow) stc_prepared();
    if (!p) return fail(STC_ENOMEM, "no host memory for the prepared setup");
    p->L = L;
    p->m = m;
    p->b = b;
    p->MP = MP;
    p->sizes.assign(L, m);
    if (g->sizes) std::copy(g->sizes, g->sizes + L, p->sizes.begin());
    try {
        p->blk.resize((size_t)L * NB * bs);
        p->diag.resize((size_t)L * bs);
    } catch (const std::bad_alloc &) {
        delete p;
        return fail(STC_ENOMEM, "no host memory for %zu packed blocks", (size_t)L * (NB + 1));
    }
    const int chunk = std::max(1, (int)std::min<size_t>(L, (64u << 20) / (NB * bs * 8)));
    const int threads = host_threads((double)L * NB * m * m * 8.0);
    BlockSource src(g);
    for (int l0 = 0; l0 < L; l0 += chunk) {
        const int l1 = std::min(L, l0 + chunk);
        LevelError lerr;
        src.load(l0 - b, l1 + b, threads, &lerr);
        if (lerr.level >= 0) rc = fail(STC_EINVAL, "%s", lerr.msg.c_str());
        if (rc == STC_OK)
            rc = pack_range(g, src, p->sizes, MP, l0, l1, threads,
                            p->blk.data() + (size_t)l0 * NB * bs, p->diag.data() + (size_t)l0 * bs);
        if (rc != STC_OK) {
            delete p;
            return rc;
        }
    }
    *out = p;
    return STC_OK;
}

stc_status stc_setup_prepared(const stc_prepared *p, const stc_options *o, stc_handle **out) {
    if (!p || !o || !out) return fail(STC_EINVAL, "null argument");
    *out = nullptr;
    // the generator as the plan sees it: its shape, dense blocks given (the
    // packed copy stands in for them; they are not read again)
    stc_generator g{};
    g.L = p->L;
    g.m = p->m;
    g.b = p->b;
    g.sizes = p->sizes.data();
    g.blocks = p->blk.data();
    Layout lay;
    stc_status rc = plan_setup(&g, o, &lay);
    if (rc != STC_OK) return rc;
    if (lay.general || lay.sparse || lay.MP != p->MP)
        return fail(STC_EINVAL, "the options ask for another storage than the prepared blocks");
    if ((rc = check_arena(o, lay)) != STC_OK) return rc;
    stc_handle *h = new_handle(&g, o, lay, p->sizes);
    const size_t bs = (size_t)lay.MP * lay.MP;
    hipError_t e = hipMemcpyAsync(h->blk64, p->blk.data(), sizeof(double) * p->blk.size(),
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->diag64, p->diag.data(), sizeof(double) * (size_t)p->L * bs,
                           hipMemcpyHostToDevice, h->stream);
    // also after a failed enqueue: the prepared blocks may be freed on return
    const hipError_t es = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) {
        delete h;
        return fail(STC_EDEVICE, "copy prepared blocks: %s", hipGetErrorString(e));
    }
    if ((rc = finish_setup(h, lay, p->b)) != STC_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return STC_OK;
}

void stc_prepared_free(stc_prepared *p) { delete p; }

void stc_destroy(stc_handle *h) { delete h; }

stc_status stc_load(stc_handle *h, const double *x, int32_t where) {
    if (!h) return fail(STC_EINVAL, "null handle");
    return load_vector(h, x, where);
}

stc_status stc_sweeps(stc_handle *h, int64_t nsweeps, double *diffs) {
    if (!h || nsweeps < 0) return fail(STC_EINVAL, "bad argument");
    const long long s0 = h->s;
    stc_status rc = run_burst(h, s0, nsweeps, 0.0);
    if (rc != STC_OK) return rc;
    h->s = s0 + nsweeps;
    if (h->stage32) h->iters32 += nsweeps;
    if (diffs && nsweeps > 1) {
        std::vector<double> ring(kRing);
        HIP_TRY(hipMemcpyAsync(ring.data(), h->st->diff, sizeof(double) * kRing,
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        for (int64_t j = 1; j < nsweeps; ++j) diffs[j - 1] = ring[(s0 + j) & kRingMask];
    }
    return STC_OK;
}

stc_status stc_profile_sweeps(stc_handle *h, int64_t nsweeps, double *ms_a, double *ms_b,
                              double *ms_fin, double *ms_sweep) {
    if (!h || nsweeps < 1) return fail(STC_EINVAL, "bad argument");
    if (flow_blocks(h) > 0) {
        // one persistent launch for the burst: its time is split evenly
        // between the two phases of each sweep
        hipEvent_t e[3];
        for (auto &x : e) HIP_TRY(hipEventCreate(&x));
        const long long s0 = h->s;
        hipError_t err = hipEventRecord(e[0], h->stream);
        if (err == hipSuccess) err = enqueue_flow(h, s0, nsweeps, 0.0);
        if (err == hipSuccess) err = hipEventRecord(e[1], h->stream);
        if (err == hipSuccess) err = end_burst(h, s0 + nsweeps, 0.0, true);
        if (err == hipSuccess) err = hipEventRecord(e[2], h->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e[2]);
        float k = 0.f, fl = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&k, e[0], e[1]);
        if (err == hipSuccess) err = hipEventElapsedTime(&fl, e[1], e[2]);
        for (auto &x : e) (void)hipEventDestroy(x);
        if (err != hipSuccess) return fail(STC_EDEVICE, "profiled sweeps: %s", hipGetErrorString(err));
        h->s = s0 + nsweeps;
        if (h->stage32) h->iters32 += nsweeps;
        if (ms_a) *ms_a = k / 2.0 / nsweeps;
        if (ms_b) *ms_b = k / 2.0 / nsweeps;
        if (ms_fin) *ms_fin = (double)fl / nsweeps;
        if (ms_sweep) *ms_sweep = ((double)k + fl) / nsweeps;
        return STC_OK;
    }
    const bool fold = folds(h);
    // per sweep: start and stop of each phase's dispatch, and around the
    // finalize launch when it is not folded; then the burst's bounds and its
    // closing flush
    std::vector<SweepTimers> tm(nsweeps);
    std::vector<hipEvent_t> ev;
    auto make = [&](hipEvent_t *e) {
        hipError_t r = hipEventCreate(e);
        if (r == hipSuccess) ev.push_back(*e);
        return r;
    };
    hipEvent_t t0 = nullptr, t1 = nullptr, fl0 = nullptr;
    hipError_t err = make(&t0);
    if (err == hipSuccess) err = make(&t1);
    if (err == hipSuccess) err = make(&fl0);
    for (auto &t : tm) {
        if (err == hipSuccess) err = make(&t.a.start);
        if (err == hipSuccess) err = make(&t.a.stop);
        if (err == hipSuccess) err = make(&t.b.start);
        if (err == hipSuccess) err = make(&t.b.stop);
        if (!fold && err == hipSuccess) err = make(&t.fin0);
        if (!fold && err == hipSuccess) err = make(&t.fin1);
    }
    auto destroy = [&]() { for (auto &e : ev) (void)hipEventDestroy(e); };
    const long long s0 = h->s;
    if (err == hipSuccess) err = hipEventRecord(t0, h->stream);
    for (int64_t j = 1; j <= nsweeps && err == hipSuccess; ++j)
        err = enqueue_sweep(h, s0 + j, 0.0, &tm[j - 1], j == 1);
    if (err == hipSuccess) err = hipEventRecord(fl0, h->stream);
    if (err == hipSuccess) err = end_burst(h, s0 + nsweeps, 0.0);
    if (err == hipSuccess) err = hipEventRecord(t1, h->stream);
    if (err == hipSuccess) err = hipEventSynchronize(t1);
    if (err != hipSuccess) {
        destroy();
        return fail(STC_EDEVICE, "profiled sweeps: %s", hipGetErrorString(err));
    }
    auto ms = [](hipEvent_t a, hipEvent_t b) {
        float x = 0.f;
        (void)hipEventElapsedTime(&x, a, b);
        return (double)x;
    };
    // Algorithm 1 sweeps in one launch: its time is phase A's, phase B's
    // events are never recorded (and not read)
    const bool two_launches = h->method == STC_STAIRCASE;
    double ta = 0.0, tb = 0.0, tf = 0.0;
    for (const auto &t : tm) {
        ta += ms(t.a.start, t.a.stop);
        if (two_launches) tb += ms(t.b.start, t.b.stop);
        if (!fold) tf += ms(t.fin0, t.fin1);
    }
    tf += ms(fl0, t1);   // the flush that ends the burst
    const double tot = ms(t0, t1);
    destroy();
    h->s = s0 + nsweeps;
    if (h->stage32) h->iters32 += nsweeps;
    if (ms_a) *ms_a = ta / nsweeps;
    if (ms_b) *ms_b = tb / nsweeps;
    if (ms_fin) *ms_fin = tf / nsweeps;
    if (ms_sweep) *ms_sweep = tot / nsweeps;
    return STC_OK;
}

int32_t stc_variant_count(void) { return variant_count(); }

stc_status stc_set_variant(stc_handle *h, int32_t stage, int32_t variant) {
    if (!h) return fail(STC_EINVAL, "null handle");
    if (stage != STC_FP64 && stage != STC_FP32) return fail(STC_EINVAL, "stage must be FP64 or FP32");
    if (variant < 0 || variant >= variant_count()) return fail(STC_EINVAL, "no variant %d", variant);
    h->variant[stage == STC_FP32 ? 1 : 0] = variant;
    return STC_OK;
}

stc_status stc_get_variant(stc_handle *h, int32_t stage, int32_t *variant) {
    if (!h || !variant) return fail(STC_EINVAL, "null argument");
    if (stage != STC_FP64 && stage != STC_FP32) return fail(STC_EINVAL, "stage must be FP64 or FP32");
    *variant = h->variant[stage == STC_FP32 ? 1 : 0];
    return STC_OK;
}

stc_status stc_autotune(stc_handle *h, int32_t trial_sweeps, double *ms_fp64, double *ms_fp32) {
    if (!h || trial_sweeps < 1) return fail(STC_EINVAL, "bad argument");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    stc_status rc = STC_OK;
    const int nv = variant_count();
    for (int stage = 0; stage < 2 && rc == STC_OK; ++stage) {
        const bool f32 = stage == 1;
        if (f32 && h->precision == STC_FP64) continue;
        if (!f32 && h->precision == STC_FP32) continue;
        // time every variant from the uniform start in this stage's precision;
        // the best per-phase variant and the best persistent one separately
        double best[2] = {1e300, 1e300};
        int best_v[2] = {-1, -1};
        // the banded sparse kernel has no variants; the any-pattern kernel has
        // its load policy (plain or non-temporal); the dense kernels all
        std::vector<int> cands;
        if (h->general || h->method == STC_JGS)
            cands = {0, 2};
        else if (h->sparse)
            cands = {h->variant[stage]};
        else
            for (int v = 0; v < nv; ++v) cands.push_back(v);
        for (int v : cands) {
            if (rc != STC_OK) break;
            if ((rc = load_vector_stage(h, nullptr, STC_MEM_HOST, f32)) != STC_OK) break;
            h->variant[stage] = v;
            if (variant_flow(v) && flow_blocks(h) == 0) continue;   // no persistent form here
            // 3 warm-up sweeps, then the timed burst, each as the solver runs them
            if ((rc = run_burst(h, 0, 3, 0.0)) != STC_OK) break;
            hipError_t e = hipEventRecord(e0, h->stream);
            if (e == hipSuccess) {
                stc_status r2 = run_burst(h, 3, trial_sweeps, 0.0);
                if (r2 != STC_OK) {
                    rc = r2;
                    break;
                }
            }
            if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = fail(STC_EDEVICE, "autotune: %s", hipGetErrorString(e));
                break;
            }
            HostState hs;
            if ((rc = read_state(h, &hs)) != STC_OK) break;   // a timed-out wait is an error
            const double per = (double)ms / trial_sweeps;
            const int kind = variant_flow(v) ? 1 : 0;
            if (per < best[kind]) {
                best[kind] = per;
                best_v[kind] = v;
            }
        }
        if (rc != STC_OK) break;
        // a persistent (cooperative) burst must beat the best per-phase
        // launches by more than kFlowMargin to be chosen: within that margin
        // the two are run-to-run noise, and plain launches ask less of the
        // device (no co-residency of the whole grid)
        constexpr double kFlowMargin = 0.02;
        const bool flow = best_v[1] >= 0 &&
                          (best_v[0] < 0 || best[1] < best[0] * (1.0 - kFlowMargin));
        h->variant[stage] = flow ? best_v[1] : (best_v[0] >= 0 ? best_v[0] : h->variant[stage]);
        const double best_ms = flow ? best[1] : best[0];
        if (f32 && ms_fp32) *ms_fp32 = best_ms;
        if (!f32 && ms_fp64) *ms_fp64 = best_ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == STC_OK) rc = load_vector(h, nullptr, STC_MEM_HOST);
    return rc;
}

stc_status stc_phase_bytes(stc_handle *h, double *bytes_a, double *bytes_b) {
    if (!h) return fail(STC_EINVAL, "null handle");
    const double sb = h->stage32 ? 4.0 : 8.0;
    const int pA = (h->stair_type == 1) ? 0 : 1;
    double out[2] = {0.0, 0.0};
    for (int ph = 0; ph < 2 && h->general; ++ph) {
        // W_i, the level's stored ELL slots (value + 4-byte index), the
        // distinct source values and the level's output
        const int par = ph == 0 ? pA : 1 - pA;
        double blocks = 0.0, vout = 0.0;
        for (int i = par; i < h->L; i += 2) {
            vout += h->sizes[i];
            blocks += (double)h->sizes[i] * h->sizes[i];
            blocks += (double)(h->gen_host[i].Kn + h->gen_host[i].Kf) * h->MP * (1.0 + 4.0 / sb);
        }
        out[ph] = sb * (blocks + h->gen_vin[ph] + vout);
    }
    for (int ph = 0; ph < 2 && !h->general; ++ph) {
        const int par = ph == 0 ? pA : 1 - pA;
        double blocks = 0.0, vin = 0.0, vout = 0.0;
        std::vector<char> seen(h->L, 0);
        for (int i = par; i < h->L; i += 2) {
            vout += h->sizes[i];
            for (int d = -h->b; d <= h->b; ++d) {
                const int k = i + d;
                if (k < 0 || k >= h->L) continue;
                // stored block: rows of level k (or i for the inverse) x columns of level i;
                // sparse storage: its slots (value + 1-byte row index) and its q_j and
                // round offsets
                if (h->sparse && d != 0) {
                    const EllShape &e = h->ell_shape[(size_t)i * h->NB + d + h->b];
                    blocks += 4.0 * (double)e.quads * (1.0 + 1.0 / sb) +
                              (e.Kq > 0 ? (double)ell_meta_bytes(h->MP, e.Kq) / sb : 0.0);
                } else
                    blocks += (double)h->sizes[k] * h->sizes[i];
                if (d != 0 && !seen[k]) {
                    seen[k] = 1;
                    vin += h->sizes[k];
                }
            }
        }
        out[ph] = sb * (blocks + vin + vout);
    }
    if (h->method == STC_JGS) {   // one launch per sweep
        out[0] += out[1];
        out[1] = 0.0;
    }
    if (bytes_a) *bytes_a = out[0];
    if (bytes_b) *bytes_b = out[1];
    return STC_OK;
}

stc_status stc_query(stc_handle *h, int64_t *sweeps, int32_t *stopped, double *diff_1) {
    if (!h) return fail(STC_EINVAL, "null handle");
    HostState hs;
    stc_status rc = read_state(h, &hs);
    if (rc != STC_OK) return rc;
    const long long cur = hs.stop_flag ? hs.stop_sweep : hs.last_sweep;
    h->s = hs.last_sweep;
    if (sweeps) *sweeps = cur;
    if (stopped) *stopped = hs.stop_flag;
    if (diff_1) {
        // latest change known for certain: at the stopped sweep, else two
        // sweeps back (batched sweeps measure it two sweeps late)
        const long long k = hs.stop_flag ? hs.stop_sweep : hs.last_sweep - 2;
        *diff_1 = INFINITY;
        if (k >= 1 && (rc = read_ring(h, h->st->diff, k, diff_1)) != STC_OK) return rc;
    }
    if (hs.status == kDevDegenerate) return fail(STC_EDEGENERATE, "e^T z <= 0 after sweep %lld", hs.stop_sweep + 1);
    return STC_OK;
}

stc_status stc_store(stc_handle *h, double *pi, int32_t where) {
    if (!h || !pi) return fail(STC_EINVAL, "null argument");
    HostState hs;
    stc_status rc = read_state(h, &hs);
    if (rc != STC_OK) return rc;
    const long long cur = hs.stop_flag ? hs.stop_sweep : hs.last_sweep;
    return store_vector(h, h->stage32, cur, pi, where);
}

stc_status stc_promote(stc_handle *h) {
    if (!h) return fail(STC_EINVAL, "null handle");
    if (!h->stage32 || h->precision == STC_FP64)
        return fail(STC_EINVAL, "the handle does not sweep in FP32");
    HostState hs;
    stc_status rc = read_state(h, &hs);
    if (rc != STC_OK) return rc;
    if (hs.status == kDevDegenerate) return fail(STC_EDEGENERATE, "e^T z <= 0");
    const long long k = hs.stop_flag ? hs.stop_sweep : hs.last_sweep;
    h->iters32 = k;
    if ((rc = widen_at(h, k)) != STC_OK) return rc;
    HIP_TRY(launch_rearm(h->st, k, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->s = k;
    return STC_OK;
}

stc_status stc_residual(stc_handle *h, const double *x, double *res_1, int32_t where) {
    if (!h || !x || !res_1) return fail(STC_EINVAL, "null argument");
    const double *src = x;
    if (where == STC_MEM_HOST) {
        HIP_TRY(hipMemcpyAsync(h->io, x, sizeof(double) * h->N, hipMemcpyHostToDevice, h->stream));
        src = h->io;
    }
    // FP64 copy in the padded layout; slot -1 = use x as given
    HIP_TRY(launch_load(8, h->MP, src, h->off, h->sizes_d, h->L, h->wres, h->part_aux,
                        (int)h->lay.naux, h->st, -1, h->stream));
    HIP_TRY(enqueue_residual(h, false, h->wres, -1));
    HostState hs;
    stc_status rc = read_state(h, &hs);
    if (rc != STC_OK) return rc;
    *res_1 = hs.residual;
    return STC_OK;
}

stc_status stc_step(stc_handle *h, const double *x, double *z, double *diff_1, int32_t where) {
    if (!h || !x || !z) return fail(STC_EINVAL, "null argument");
    if (x == z) return fail(STC_EINVAL, "z may not alias x");
    stc_status rc = load_vector(h, x, where);
    if (rc != STC_OK) return rc;
    if ((rc = run_burst(h, 0, 1, 0.0)) != STC_OK) return rc;   // records sweep 1 and its change
    h->s = 1;
    if (h->stage32) h->iters32 = 1;
    HostState hs;
    if ((rc = read_state(h, &hs)) != STC_OK) return rc;
    if (hs.status == kDevDegenerate) return fail(STC_EDEGENERATE, "e^T z <= 0");
    if (diff_1 && (rc = read_ring(h, h->st->diff, 1, diff_1)) != STC_OK) return rc;
    return store_vector(h, h->stage32, 1, z, where);
}

stc_status stc_solve(stc_handle *h, const double *x0, double tol, int64_t maxit, double *pi,
                     stc_result *res, int32_t where) {
    if (!h || !pi) return fail(STC_EINVAL, "null argument");
    if (maxit < 0 || !(tol >= 0.0)) return fail(STC_EINVAL, "need maxit >= 0 and tol >= 0");
    stc_status rc = load_vector(h, x0, where);
    if (rc != STC_OK) return rc;
    const bool mixed = h->precision == STC_MIXED;
    auto device_tol = [&]() {
        if (mixed && h->stage32) return h->switch_tol;
        return h->stop == STC_STOP_DIFF ? tol : 0.0;
    };
    long long s = 0, final_k = -1;
    bool converged = false;
    HostState hs;
    // The FP32 stage also ends at its rounding floor, which may lie above
    // switch_tol: its change is read every kStallSweeps sweeps (or every
    // burst, if longer), and after kStallReads readings in a row with no new
    // low the solve continues in FP64 from the current sweep.  A converging
    // stage makes a new low at every reading.
    constexpr long long kStallSweeps = 32;
    constexpr int kStallReads = 4;
    long long next_read = 0;
    double low32 = INFINITY;
    int stale = 0;
    auto to_fp64 = [&](long long k) -> stc_status {
        h->iters32 = k;
        stc_status r = widen_at(h, k);
        if (r != STC_OK) return r;
        HIP_TRY(launch_rearm(h->st, k, h->stream));
        s = k;
        h->s = k;
        return STC_OK;
    };
    while (s < maxit) {
        const long long n = std::min<long long>(h->check_every, maxit - s);
        const double dt = device_tol();
        if ((rc = run_burst(h, s, n, dt)) != STC_OK) return rc;
        s += n;
        h->s = s;
        if ((rc = read_state(h, &hs)) != STC_OK) return rc;
        if (hs.status == kDevDegenerate) {
            final_k = hs.stop_sweep;
            rc = fail(STC_EDEGENERATE, "e^T z <= 0 after sweep %lld", hs.stop_sweep + 1);
            store_vector(h, h->stage32, final_k, pi, where);
            if (res) { res->iters = final_k; res->status = rc; }
            return rc;
        }
        if (hs.stop_flag) {
            const long long k = hs.stop_sweep;
            if (mixed && h->stage32) {
                // FP32 stage done: continue in FP64 from sweep k
                if ((rc = to_fp64(k)) != STC_OK) return rc;
                continue;
            }
            final_k = k;
            converged = true;
            break;
        }
        if (mixed && h->stage32 && s >= next_read && s < maxit) {
            next_read = s + std::max<long long>(h->check_every, kStallSweeps);
            double d;
            if ((rc = read_ring(h, h->st->diff, s, &d)) != STC_OK) return rc;
            if (d < low32) {
                low32 = d;
                stale = 0;
            } else if (++stale >= kStallReads) {
                // FP32 rounding floor: continue in FP64 from sweep s
                if ((rc = to_fp64(s)) != STC_OK) return rc;
                continue;
            }
        }
        if (h->stop == STC_STOP_RESIDUAL && !(mixed && h->stage32)) {
            double r;
            if ((rc = residual_of(h, h->stage32, s, &r)) != STC_OK) return rc;
            if (r <= tol) {
                final_k = s;
                converged = true;
                break;
            }
        }
    }
    if (final_k < 0) final_k = s;   // maxit reached
    if (h->stage32) h->iters32 = final_k;   // ended in FP32 (also a mixed solve at maxit)
    h->s = final_k;
    double diff = INFINITY;   // every burst ends with the changes up to its last sweep
    if (final_k >= 1 && (rc = read_ring(h, h->st->diff, final_k, &diff)) != STC_OK) return rc;
    double r;
    if ((rc = residual_of(h, h->stage32, final_k, &r)) != STC_OK) return rc;
    if (!converged) converged = (h->stop == STC_STOP_DIFF) ? (diff <= tol) : (r <= tol);
    if ((rc = store_vector(h, h->stage32, final_k, pi, where)) != STC_OK) return rc;
    const stc_status out = converged ? STC_OK : fail(STC_EMAXIT, "maxit = %lld sweeps done, "
                                                     "stop quantity above tol", (long long)maxit);
    if (res) {
        res->residual_1 = r;
        res->diff_1 = diff;
        res->iters = final_k;
        res->iters_fp32 = mixed ? h->iters32 : (h->precision == STC_FP32 ? final_k : 0);
        res->status = out;
    }
    return out;
}

stc_status stc_solve_gmres(stc_handle *h, const double *x0, int32_t restart, double tol,
                           int64_t max_applies, double *pi, stc_result *res, int32_t where) {
    if (!h || !pi) return fail(STC_EINVAL, "null argument");
    if (h->kr < 1) return fail(STC_EINVAL, "the handle has no Krylov workspace (krylov_restart = 0)");
    if (h->method != STC_STAIRCASE) return fail(STC_EINVAL, "GMRES takes the stair splitting");
    if (restart < 1 || restart > h->kr)
        return fail(STC_EINVAL, "restart must be in 1..%d (krylov_restart)", h->kr);
    if (max_applies < 2 || !(tol >= 0.0)) return fail(STC_EINVAL, "need max_applies >= 2 and tol >= 0");
    const size_t n = (size_t)h->L * h->MP;
    const int G = kDotGroups;
    const int r = restart;
    double *X = h->kX, *W = h->kW, *V = h->kV;
    // device scalars, y, then per step j: ||w_j|| and the coefficients of
    // both passes (columns of r + 2), so a cycle needs no host round trip
    // until its end
    double *scal = h->kh, *ydev = h->kh + 8, *knorm = ydev + r, *H1 = knorm + r,
           *H2 = H1 + (size_t)r * (r + 2);
    hipStream_t st = h->stream;
    // x = x0 / e^T x0 (checked like any start vector), in the Krylov x buffer
    stc_status rc = load_vector_stage(h, x0, where, false);
    if (rc != STC_OK) return rc;
    HIP_TRY(launch_kscale((const double *)wbuf(h, false, 0), &h->st->x_sum, X, n, st));
    auto residual = [&](double *out) -> stc_status {
        HIP_TRY(enqueue_residual(h, false, X, -1));
        HostState hs;
        stc_status r2 = read_state(h, &hs);
        if (r2 == STC_OK) *out = hs.residual;
        return r2;
    };
    auto fetch = [&](const double *src, double *dst, size_t count) -> stc_status {
        HIP_TRY(hipMemcpyAsync(dst, src, sizeof(double) * count, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        return STC_OK;
    };
    double res1;
    if ((rc = residual(&res1)) != STC_OK) return rc;
    long long applies = 0, applies32 = 0;
    double diff = INFINITY;
    bool converged = res1 <= tol, stalled = false;
    // FP32 and mixed handles apply M^{-1} N in FP32 first (the Krylov vectors
    // stay FP64), until ||Q^T x||_1 <= switch_tol or an FP32 cycle stalls
    bool f32 = h->precision != STC_FP64;
    auto apply = [&](const double *v, double *o) -> hipError_t {
        ++applies;
        if (f32) ++applies32;
        return enqueue_apply(h, v, o, f32);
    };
    std::vector<double> R((size_t)r * r), cs(r), sn(r), g(r + 1), y(r);
    std::vector<double> hv((size_t)r + 2 * (size_t)r * (r + 2));
    // safeguard: a cycle is kept only if it lowers ||Q^T x||_1 per
    // application of T by at least the square of the factor of the last
    // block of plain steps (before any: by half over the cycle); otherwise x
    // stays and k plain applications of T follow (k = restart at first,
    // doubled after every rejected cycle)
    constexpr int kNormEvery = 16;
    long long k_plain = r;
    double plain_rate = -1.0;   // none measured yet
    while (!converged && applies + 2 <= max_applies) {
        const int rr = (int)std::min<long long>(r, max_applies - applies - 1);
        // v_0 = (T x - x) / beta
        HIP_TRY(apply(X, W));
        HIP_TRY(launch_kaxpby(1.0, W, -1.0, X, V, n, st));
        HIP_TRY(launch_kdots(V, n, 1, V, n, h->kdot, G, scal, true, st));
        double beta;
        if ((rc = fetch(scal, &beta, 1)) != STC_OK) return rc;
        if (!(beta > 0.0) || !std::isfinite(beta)) {
            // T x = x to rounding (or the FP32 apply overflowed): no Krylov
            // direction is left in this precision.  An FP32 stage ends and the
            // FP64 cycles take over; in FP64 the solve stops, and the status
            // below compares the residual with tol.
            if (f32) {
                f32 = false;
                continue;
            }
            stalled = true;
            break;
        }
        HIP_TRY(launch_kscale(V, scal, V, n, st));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        // the Arnoldi steps of the cycle, enqueued without a host round trip
        for (int j = 0; j < rr; ++j) {
            double *vj = V + (size_t)j * n;
            double *h1 = H1 + (size_t)j * (r + 2), *h2 = H2 + (size_t)j * (r + 2);
            // w = v_j - T v_j = B v_j, orthogonalised against v_0 .. v_j twice
            HIP_TRY(apply(vj, W));
            HIP_TRY(launch_kaxpby(1.0, vj, -1.0, W, W, n, st));
            HIP_TRY(launch_kdots(V, n, j + 1, W, n, h->kdot, G, h1, false, st));
            HIP_TRY(launch_kupdate(V, n, j + 1, h1, -1.0, W, n, st));
            HIP_TRY(launch_kdots(V, n, j + 1, W, n, h->kdot, G, h2, false, st));
            HIP_TRY(launch_kupdate(V, n, j + 1, h2, -1.0, W, n, st));
            HIP_TRY(launch_kdots(W, n, 1, W, n, h->kdot, G, knorm + j, true, st));
            // v_{j+1} = w / ||w||; after a breakdown (||w|| = 0) this and the
            // later vectors are not finite, and the least-squares step below
            // stops before them
            HIP_TRY(launch_kscale(W, knorm + j, V + (size_t)(j + 1) * n, n, st));
        }
        // the cycle's Hessenberg columns, rotated on the host
        if ((rc = fetch(knorm, hv.data(), (size_t)r + (size_t)r * (r + 2) + (size_t)rr * (r + 2))) !=
            STC_OK)
            return rc;
        const double *hn_h = hv.data(), *H1h = hv.data() + r, *H2h = H1h + (size_t)r * (r + 2);
        int used = 0;
        for (int j = 0; j < rr; ++j) {
            std::vector<double> c(j + 2);
            bool finite = std::isfinite(hn_h[j]);
            for (int i = 0; i <= j; ++i) {
                c[i] = H1h[(size_t)j * (r + 2) + i] + H2h[(size_t)j * (r + 2) + i];
                finite = finite && std::isfinite(c[i]);
            }
            if (!finite) break;
            c[j + 1] = hn_h[j];
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * c[i] + sn[i] * c[i + 1];
                c[i + 1] = -sn[i] * c[i] + cs[i] * c[i + 1];
                c[i] = t;
            }
            const double nr = std::hypot(c[j], c[j + 1]);
            if (nr == 0.0) break;
            cs[j] = c[j] / nr;
            sn[j] = c[j + 1] / nr;
            c[j] = nr;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            for (int i = 0; i <= j; ++i) R[(size_t)i * r + j] = c[i];
            used = j + 1;
            // a breakdown (the Krylov space holds the solution), or the
            // estimate at the rounding floor: the later columns add nothing
            if (!(hn_h[j] > 1e-300) || std::fabs(g[j + 1]) <= 1e-15 * beta) break;
        }
        if (used == 0) break;
        // R y = g (upper triangular), then x += V y, normalised
        for (int i = used - 1; i >= 0; --i) {
            double t = g[i];
            for (int k = i + 1; k < used; ++k) t -= R[(size_t)i * r + k] * y[k];
            y[i] = R[(size_t)i * r + i] != 0.0 ? t / R[(size_t)i * r + i] : 0.0;
        }
        HIP_TRY(hipMemcpyAsync(ydev, y.data(), sizeof(double) * used, hipMemcpyHostToDevice, st));
        HIP_TRY(launch_kaxpby(1.0, X, 0.0, X, W, n, st));   // the previous x
        HIP_TRY(launch_kupdate(V, n, used, ydev, 1.0, X, n, st));
        HIP_TRY(launch_kdots(X, n, 1, nullptr, n, h->kdot, G, scal + 1, false, st));
        double sum;
        if ((rc = fetch(scal + 1, &sum, 1)) != STC_OK) return rc;
        // normalise by any finite non-zero sum (a step that flips the sign of
        // the null-space component still gives the normalised vector); a
        // zero or non-finite sum makes the cycle a rejected one
        double res_new = INFINITY;
        if (sum != 0.0 && std::isfinite(sum)) {
            HIP_TRY(launch_kscale(X, scal + 1, X, n, st));
            if ((rc = residual(&res_new)) != STC_OK) return rc;
        } else {
            HIP_TRY(launch_kaxpby(1.0, W, 0.0, W, X, n, st));
        }
        const int cyc_applies = rr + 1;   // every step of the cycle ran
        const double need = plain_rate < 0.0 ? std::pow(0.5, 1.0 / cyc_applies)
                                             : plain_rate * plain_rate;
        if (h->keep_all && !std::isfinite(res_new)) {
            rc = fail(STC_EDEGENERATE, "a GMRES cycle gave e^T x = %g", sum);
            if (res) {
                res->iters = applies;
                res->status = rc;
            }
            return rc;
        }
        const bool keep = h->keep_all ||
                          (std::isfinite(res_new) && res_new < res1 &&
                           std::pow(res_new / res1, 1.0 / cyc_applies) <= need);
        if (f32 && (!keep || res_new <= h->switch_tol)) {
            // the FP32 stage ends: at its rounding floor, a stalled cycle is
            // dropped; the FP64 cycles continue from the best x
            f32 = false;
            if (keep) {
                HIP_TRY(launch_kdots(X, n, 1, W, n, h->kdot, G, scal + 2, false, st, true));
                if ((rc = fetch(scal + 2, &diff, 1)) != STC_OK) return rc;
                res1 = res_new;
            } else {
                HIP_TRY(launch_kaxpby(1.0, W, 0.0, W, X, n, st));
            }
        } else if (keep) {
            HIP_TRY(launch_kdots(X, n, 1, W, n, h->kdot, G, scal + 2, false, st, true));
            if ((rc = fetch(scal + 2, &diff, 1)) != STC_OK) return rc;
            res1 = res_new;
        } else {
            // keep the previous x and take plain steps x <- T x from it
            HIP_TRY(launch_kaxpby(1.0, W, 0.0, W, X, n, st));
            const long long steps = std::min<long long>(k_plain, max_applies - applies);
            if (steps > 0) {
                HIP_TRY(launch_kaxpby(1.0, X, 0.0, X, V, n, st));   // for the change
                double *src = X, *dstv = W;
                for (long long t = 0; t < steps; ++t) {
                    HIP_TRY(apply(src, dstv));
                    std::swap(src, dstv);
                    if ((t + 1) % kNormEvery == 0) {
                        HIP_TRY(launch_kdots(src, n, 1, nullptr, n, h->kdot, G, scal + 3, false, st));
                        HIP_TRY(launch_kscale(src, scal + 3, src, n, st));
                    }
                }
                if (src != X) HIP_TRY(launch_kaxpby(1.0, src, 0.0, src, X, n, st));
                HIP_TRY(launch_kdots(X, n, 1, nullptr, n, h->kdot, G, scal + 1, false, st));
                if ((rc = fetch(scal + 1, &sum, 1)) != STC_OK) return rc;
                if (!(sum > 0.0) || !std::isfinite(sum)) {
                    rc = fail(STC_EDEGENERATE, "e^T x = %g after plain steps", sum);
                    if (res) {
                        res->iters = applies;
                        res->status = rc;
                    }
                    return rc;
                }
                HIP_TRY(launch_kscale(X, scal + 1, X, n, st));
                HIP_TRY(launch_kdots(X, n, 1, V, n, h->kdot, G, scal + 2, false, st, true));
                if ((rc = fetch(scal + 2, &diff, 1)) != STC_OK) return rc;
                double res_plain;
                if ((rc = residual(&res_plain)) != STC_OK) return rc;
                plain_rate = res1 > 0.0 ? std::pow(res_plain / res1, 1.0 / (double)steps) : 1.0;
                res1 = res_plain;
            }
            k_plain = std::min<long long>(2 * k_plain, max_applies);
        }
        converged = res1 <= tol;
    }
    // pi = x (the apply-state's scales are 1)
    double *dst = (where == STC_MEM_DEVICE) ? pi : h->io;
    HIP_TRY(launch_store(8, h->MP, X, h->off, h->sizes_d, h->L, h->kst, 0, dst, st));
    if (where == STC_MEM_HOST)
        HIP_TRY(hipMemcpyAsync(pi, h->io, sizeof(double) * h->N, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const stc_status out =
        converged ? STC_OK
        : stalled ? fail(STC_EMAXIT, "GMRES stalled: T x = x to rounding at residual %g above tol", res1)
                  : fail(STC_EMAXIT, "max_applies = %lld reached, residual %g above tol",
                         (long long)max_applies, res1);
    if (res) {
        res->residual_1 = res1;
        res->diff_1 = diff;
        res->iters = applies;
        res->iters_fp32 = applies32;
        res->status = out;
    }
    return out;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched sweeps over many chains
// ---------------------------------------------------------------------------

constexpr int kSizeClasses = 5;                       // MP = 8, 16, 32, 64, 128
constexpr int kCountsPerGroup = 1 + 6 * kSizeClasses;
// Index, within a stage group's counts, of size class c's entry k: 0 and 1
// phase A {offset, count} into the work list, 2 and 3 phase B's, 4 and 5
// {offset, count} of the class's chains in the group's chain table.
constexpr int cnt_at(int c, int k) { return 1 + 6 * c + k; }

// Launch shape of the batched kernel for one (precision stage, padded block
// size): the tile (launch variant bits 0 and 1: row groups per level,
// non-temporal loads), the groups of levels per work item and the
// persistent grid in workgroups per compute unit.  Untuned: variant 0 with
// the batch's load policy, one group per item, 8 workgroups per CU.
struct BatchTile {
    bool tuned = false;
    int variant = 0;
    int per_item = 1;
    int grid_per_cu = 8;
};

struct stc_batch {
    int max_chains = 0;
    long long max_items = 0;
    int b = 1;
    bool nt = false;
    double tol = 0.0;    // change tolerance of the last stc_batch_set
    int cus = 256;       // compute units of the device
    BatchTile tile[2][kSizeClasses];   // [stage: 0 FP64, 1 FP32][size class: MP = 8 << c]
    hipStream_t stream = nullptr;
    bool own_stream = false;   // created here: graph capture needs a non-null stream
    // each (stage group, block size) present runs its two phases on a side
    // stream of its own, forked from the batch's stream and joined back, so
    // the launches of different block sizes overlap
    hipStream_t side[2 * kSizeClasses] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[2 * kSizeClasses] = {};
    char *base = nullptr;
    ChainDesc *d_chains[2] = {nullptr, nullptr};   // [0] FP64 stage, [1] FP32 stage
    WorkItem *d_items_a[2] = {nullptr, nullptr};
    WorkItem *d_items_b[2] = {nullptr, nullptr};
    // per stage group g (kCountsPerGroup ints from g * kCountsPerGroup):
    // chains, then per block size class c (MP = 8 << c): phase A {offset,
    // count}, phase B {offset, count} into that group's work lists, and the
    // class's {offset, count} in the group's chain table (ordered by class)
    int *d_counts = nullptr;
    int counts[2 * kCountsPerGroup] = {};
    DevState **d_states = nullptr;                  // members' states, in stc_batch_set order
    QueryRow *d_query = nullptr;
    std::vector<stc_handle *> members;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    long long graph_n = -1;
    int graph_groups = -1;
};

namespace {

struct BatchLayout {
    size_t chains = 0, items_a = 0, items_b = 0, counts = 0, states = 0, query = 0, total = 0;
};

BatchLayout batch_layout(int max_chains, long long max_items) {
    BatchLayout l;
    size_t at = 0;
    auto take = [&](size_t bytes) { size_t p = at; at = align_up(at + bytes); return p; };
    l.chains = take(2 * (size_t)max_chains * sizeof(ChainDesc));
    l.items_a = take(2 * (size_t)max_items * sizeof(WorkItem));
    l.items_b = take(2 * (size_t)max_items * sizeof(WorkItem));
    l.counts = take(2 * kCountsPerGroup * sizeof(int));
    l.states = take((size_t)max_chains * sizeof(DevState *));
    l.query = take((size_t)max_chains * sizeof(QueryRow));
    l.total = at;
    return l;
}

// Release the captured graph.  Its last launch may still be queued or
// running on the batch's stream (stc_batch_sweeps returns at once), so the
// stream drains first.
void drop_graph(stc_batch *bt) {
    if (bt->exec) (void)hipStreamSynchronize(bt->stream);
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    bt->exec = nullptr;
    bt->graph = nullptr;
    bt->graph_n = -1;
    bt->graph_groups = -1;
}

int class_of(int MP) {
    int c = 0;
    while ((8 << c) < MP) ++c;
    return c;
}

// Launch variant of the batched kernel for stage group g and size class c.
int tile_variant(const stc_batch *bt, int g, int c) {
    const BatchTile &t = bt->tile[g][c];
    return t.tuned ? t.variant : (bt->nt ? 2 : 0);
}

// Build the chain table and the work lists of the batch's members on the
// device, with change tolerance tol (timing: every stopping test off), and
// give each member the batch's launch variant for its block size in both
// stages (so the chain swept alone takes the same per-level arithmetic).
stc_status upload_lists(stc_batch *bt, double tol, bool timing = false) {
    const int count = (int)bt->members.size();
    std::vector<ChainDesc> chains[2];
    // work lists per stage group and block size class, in chain order; the
    // chain table of each group holds the chains class by class
    std::vector<WorkItem> ia[2][kSizeClasses], ib[2][kSizeClasses];
    // phase A lists start with one reduction item per chain (dispatched
    // first, so they run beside the streaming items)
    std::vector<WorkItem> fold_a[2][kSizeClasses];
    std::vector<int> order;
    for (int cls = 0; cls < kSizeClasses; ++cls)
        for (int c = 0; c < count; ++c)
            if (class_of(bt->members[c]->MP) == cls) order.push_back(c);
    int cls_first[2][kSizeClasses], cls_count[2][kSizeClasses] = {};
    for (int c : order) {
        stc_handle *h = bt->members[c];
        const int g = h->stage32 ? 1 : 0;
        const int bytes = g == 1 ? 4 : 8;
        const int cls = class_of(h->MP);
        const int v = tile_variant(bt, g, cls);
        h->variant[0] = tile_variant(bt, 0, cls);
        h->variant[1] = tile_variant(bt, 1, cls);
        const int pA = (h->stair_type == 1) ? 0 : 1;
        ChainDesc d;
        d.blk = g == 1 ? (const void *)h->blk32 : (const void *)h->blk64;
        for (int k = 0; k < 4; ++k) d.w[k] = wbuf(h, g == 1, k);
        d.part_sum = h->part_sum;
        d.part_diff = h->part_diff;
        d.st = h->st;
        d.L = h->L;
        d.MP = h->MP;
        d.parity_a = pA;
        d.groups_a = phase_groups(bytes, h->MP, h->L, pA, v);
        d.groups_b = phase_groups(bytes, h->MP, h->L, 1 - pA, v);
        d.nparts = (int)h->lay.nparts;
        d.tol = timing ? 0.0 : (g == 1 && h->precision == STC_MIXED) ? h->switch_tol : tol;
        const int ci = (int)chains[g].size();
        if (cls_count[g][cls]++ == 0) cls_first[g][cls] = ci;
        chains[g].push_back(d);
        const int per = bt->tile[g][cls].per_item;
        fold_a[g][cls].push_back({ci, -1, 0});
        for (int q = 0; q < d.groups_a; q += per)
            ia[g][cls].push_back({ci, q, std::min(per, d.groups_a - q)});
        for (int q = 0; q < d.groups_b; q += per)
            ib[g][cls].push_back({ci, q, std::min(per, d.groups_b - q)});
    }
    // every host table is built (and checked) before the first copy, and
    // lives until the copies are done: hipMemcpyAsync reads its host source
    // until the copy completes
    std::vector<WorkItem> lists[2][2];   // [stage group][phase]
    int counts[2 * kCountsPerGroup] = {};
    for (int g = 0; g < 2; ++g) {
        int *hc = counts + g * kCountsPerGroup;
        hc[0] = (int)chains[g].size();
        for (int ph = 0; ph < 2; ++ph) {
            std::vector<WorkItem> &all = lists[g][ph];
            for (int c = 0; c < kSizeClasses; ++c) {
                const std::vector<WorkItem> &items = ph == 0 ? ia[g][c] : ib[g][c];
                hc[cnt_at(c, 2 * ph)] = (int)all.size();       // offset
                hc[cnt_at(c, 2 * ph + 1)] =                    // count
                    (int)((ph == 0 ? fold_a[g][c].size() : 0) + items.size());
                hc[cnt_at(c, 4)] = cls_count[g][c] ? cls_first[g][c] : 0;
                hc[cnt_at(c, 5)] = cls_count[g][c];
                if (ph == 0) all.insert(all.end(), fold_a[g][c].begin(), fold_a[g][c].end());
                all.insert(all.end(), items.begin(), items.end());
            }
            if ((long long)all.size() > bt->max_items)
                return fail(STC_EINVAL, "work list of %zu items exceeds max_items %lld", all.size(),
                            bt->max_items);
        }
    }
    std::vector<DevState *> states(count);
    for (int c = 0; c < count; ++c) states[c] = bt->members[c]->st;
    std::copy(counts, counts + 2 * kCountsPerGroup, bt->counts);
    hipError_t e = hipSuccess;
    for (int g = 0; g < 2 && e == hipSuccess; ++g) {
        for (int ph = 0; ph < 2 && e == hipSuccess; ++ph)
            if (!lists[g][ph].empty())
                e = hipMemcpyAsync(ph == 0 ? bt->d_items_a[g] : bt->d_items_b[g],
                                   lists[g][ph].data(), lists[g][ph].size() * sizeof(WorkItem),
                                   hipMemcpyHostToDevice, bt->stream);
        if (e == hipSuccess && !chains[g].empty())
            e = hipMemcpyAsync(bt->d_chains[g], chains[g].data(),
                               chains[g].size() * sizeof(ChainDesc), hipMemcpyHostToDevice,
                               bt->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(bt->d_counts, bt->counts, sizeof(bt->counts), hipMemcpyHostToDevice,
                           bt->stream);
    if (e == hipSuccess && count > 0)
        e = hipMemcpyAsync(bt->d_states, states.data(), sizeof(DevState *) * count,
                           hipMemcpyHostToDevice, bt->stream);
    // also after a failed enqueue: the copies already queued read the tables
    const hipError_t es = hipStreamSynchronize(bt->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return fail(STC_EDEVICE, "batch tables: %s", hipGetErrorString(e));
    return STC_OK;
}

// Enqueue n sweeps of every non-empty stage group.  Each (stage group,
// block size) present runs its n sweeps on a side stream of its own, forked
// from the batch's stream once and joined back once: no chain depends on a
// chain of another block size, so the branches need not meet between
// sweeps, and each branch's launch gaps are filled by the others' work.  A
// branch numbers its chains' sweeps from their last recorded one, runs phase
// A (whose reduction items record each chain's previous sweep) and phase B
// per sweep, and a finalize launch records the burst's last sweep.
// Captured, the burst is a graph with one chain of launches per branch; the
// per-chain arithmetic does not depend on how the branches interleave.
hipError_t enqueue_batch(stc_batch *bt, long long n) {
    hipError_t e = hipEventRecord(bt->fork, bt->stream);
    for (int g = 1; g >= 0 && e == hipSuccess; --g) {
        const int *hc = bt->counts + g * kCountsPerGroup;
        int *dc = bt->d_counts + g * kCountsPerGroup;
        if (hc[0] == 0) continue;
        const int bytes = g == 1 ? 4 : 8;
        for (int c = 0; c < kSizeClasses && e == hipSuccess; ++c) {
            if (hc[cnt_at(c, 5)] == 0) continue;   // absent
            const int br = g * kSizeClasses + c;
            hipStream_t sc = bt->side[br];
            e = hipStreamWaitEvent(sc, bt->fork, 0);
            if (e == hipSuccess)
                e = launch_batch_begin(bt->max_chains, bt->d_chains[g], dc + cnt_at(c, 4), sc);
            const BatchTile &t = bt->tile[g][c];
            for (long long j = 0; j < n && e == hipSuccess; ++j) {
                for (int ph = 0; ph < 2 && e == hipSuccess; ++ph) {
                    if (hc[cnt_at(c, 2 * ph + 1)] == 0) continue;
                    e = launch_batch_phase(bytes, bt->b, 8 << c, ph == 1, tile_variant(bt, g, c),
                                           t.grid_per_cu * bt->cus, bt->d_chains[g],
                                           ph == 0 ? bt->d_items_a[g] : bt->d_items_b[g],
                                           dc + cnt_at(c, 2 * ph), (int)j, sc);
                }
            }
            if (e == hipSuccess)
                e = launch_batch_finalize(bt->max_chains, bt->d_chains[g], dc + cnt_at(c, 4),
                                          (int)(n - 1), sc);
            if (e == hipSuccess) e = hipEventRecord(bt->join[br], sc);
            if (e == hipSuccess) e = hipStreamWaitEvent(bt->stream, bt->join[br], 0);
        }
    }
    return e;
}

// Side streams and events of a batch; false (all released) on failure.
bool make_branches(stc_batch *bt) {
    bool ok = hipEventCreateWithFlags(&bt->fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < 2 * kSizeClasses && ok; ++k)
        ok = hipStreamCreateWithFlags(&bt->side[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&bt->join[k], hipEventDisableTiming) == hipSuccess;
    return ok;
}

void free_branches(stc_batch *bt) {
    for (int k = 0; k < 2 * kSizeClasses; ++k) {
        if (bt->side[k]) {
            (void)hipStreamSynchronize(bt->side[k]);
            (void)hipStreamDestroy(bt->side[k]);
        }
        if (bt->join[k]) (void)hipEventDestroy(bt->join[k]);
        bt->side[k] = nullptr;
        bt->join[k] = nullptr;
    }
    if (bt->fork) (void)hipEventDestroy(bt->fork);
    bt->fork = nullptr;
}

// Which (stage group, block size) launches a captured graph holds.
int batch_shape(const stc_batch *bt) {
    int mask = 0;
    for (int g = 0; g < 2; ++g)
        for (int c = 0; c < kSizeClasses; ++c)
            if (bt->counts[g * kCountsPerGroup + cnt_at(c, 5)] > 0)
                mask |= 1 << (g * kSizeClasses + c);
    return mask;
}

}  // namespace

extern "C" {

size_t stc_batch_footprint(int32_t max_chains, int64_t max_items) {
    if (max_chains < 1 || max_items < 1) return 0;
    return batch_layout(max_chains, max_items).total;
}

stc_status stc_batch_create(int32_t max_chains, int64_t max_items, int32_t b, void *stream,
                            void *arena, size_t arena_bytes, stc_batch **out) {
    if (!out) return fail(STC_EINVAL, "null argument");
    *out = nullptr;
    if (max_chains < 1 || max_items < 1 || b < 1 || b > kMaxBandwidth)
        return fail(STC_EINVAL, "need max_chains >= 1, max_items >= 1, b in 1..4");
    if (!arena || (uintptr_t)arena % kAlign) return fail(STC_EINVAL, "arena must be 256-byte aligned");
    const BatchLayout l = batch_layout(max_chains, max_items);
    if (arena_bytes < l.total)
        return fail(STC_ENOMEM, "batch arena holds %zu bytes, %zu needed", arena_bytes, l.total);
    stc_batch *bt = new stc_batch();
    bt->max_chains = max_chains;
    bt->max_items = max_items;
    bt->b = b;
    bt->stream = (hipStream_t)stream;
    if (!bt->stream) {
        if (hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking) != hipSuccess) {
            delete bt;
            return fail(STC_EDEVICE, "could not create the batch stream");
        }
        bt->own_stream = true;
    }
    bt->base = (char *)arena;
    for (int g = 0; g < 2; ++g) {
        bt->d_chains[g] = (ChainDesc *)(bt->base + l.chains) + (size_t)g * max_chains;
        bt->d_items_a[g] = (WorkItem *)(bt->base + l.items_a) + (size_t)g * max_items;
        bt->d_items_b[g] = (WorkItem *)(bt->base + l.items_b) + (size_t)g * max_items;
    }
    bt->d_counts = (int *)(bt->base + l.counts);
    bt->d_states = (DevState **)(bt->base + l.states);
    bt->d_query = (QueryRow *)(bt->base + l.query);
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    bt->cus = cus;   // persistent grids are multiples of it; workgroups without work exit
    if (!make_branches(bt)) {
        free_branches(bt);
        if (bt->own_stream) (void)hipStreamDestroy(bt->stream);
        delete bt;
        return fail(STC_EDEVICE, "could not create the batch's side streams");
    }
    hipError_t e = hipMemcpyAsync(bt->d_counts, bt->counts, sizeof(bt->counts),
                                  hipMemcpyHostToDevice, bt->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(bt->stream);
    if (e != hipSuccess) {
        free_branches(bt);
        if (bt->own_stream) (void)hipStreamDestroy(bt->stream);
        delete bt;
        return fail(STC_EDEVICE, "batch create: %s", hipGetErrorString(e));
    }
    *out = bt;
    return STC_OK;
}

stc_status stc_batch_set(stc_batch *bt, stc_handle *const *hs, int32_t count, double tol,
                         int32_t nontemporal) {
    if (!bt || (count > 0 && !hs) || count < 0) return fail(STC_EINVAL, "bad argument");
    if (count > bt->max_chains) return fail(STC_EINVAL, "%d chains > max_chains %d", count, bt->max_chains);
    for (int c = 0; c < count; ++c) {
        stc_handle *h = hs[c];
        if (!h) return fail(STC_EINVAL, "handle %d is NULL", c);
        if (h->b != bt->b) return fail(STC_EINVAL, "handle %d has bandwidth %d, batch %d", c, h->b, bt->b);
        if (h->sparse) return fail(STC_EINVAL, "handle %d stores sparse blocks; batches take dense chains", c);
        if (h->method != STC_STAIRCASE)
            return fail(STC_EINVAL, "handle %d sweeps Algorithm 1; batches take the stair splitting", c);
    }
    const bool nt = nontemporal != 0;
    if (nt != bt->nt) drop_graph(bt);
    bt->nt = nt;
    bt->tol = tol;
    bt->members.assign(hs, hs + count);
    const stc_status rc = upload_lists(bt, tol);
    if (rc != STC_OK) {
        // leave a consistent, empty batch (the device tables of the earlier
        // members are not kept beside a member list they do not match)
        bt->members.clear();
        std::string why = stc_last_error();
        (void)upload_lists(bt, tol);
        return fail(rc, "%s", why.c_str());
    }
    return STC_OK;
}

stc_status stc_batch_autotune(stc_batch *bt, int32_t trial_sweeps, double *ms_per_sweep) {
    if (!bt || trial_sweeps < 1) return fail(STC_EINVAL, "bad argument");
    if (bt->members.empty()) return fail(STC_EINVAL, "the batch has no chains to tune on");
    drop_graph(bt);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // time the whole batch (stopping tests off) with the current tiles
    auto timed = [&](double *ms) -> stc_status {
        stc_status r = upload_lists(bt, 0.0, true);
        if (r != STC_OK) return r;
        HIP_TRY(enqueue_batch(bt, 2));
        HIP_TRY(hipEventRecord(e0, bt->stream));
        HIP_TRY(enqueue_batch(bt, trial_sweeps));
        HIP_TRY(hipEventRecord(e1, bt->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        *ms = (double)t / trial_sweeps;
        return STC_OK;
    };
    stc_status rc = upload_lists(bt, 0.0, true);
    double best_ms = INFINITY;
    // one (stage, block size) at a time, the others at their current shape,
    // on the whole batch's time (the branches of different sizes overlap)
    for (int g = 0; g < 2 && rc == STC_OK; ++g)
        for (int c = 0; c < kSizeClasses && rc == STC_OK; ++c) {
            if (bt->counts[g * kCountsPerGroup + cnt_at(c, 5)] == 0) continue;   // absent
            const int MP = 8 << c;
            BatchTile best = bt->tile[g][c];
            best.variant = tile_variant(bt, g, c);
            best.tuned = true;
            double best_c = INFINITY;
            for (int v = 0; v < 4 && rc == STC_OK; ++v) {
                // variants that differ only in row groups the block size ignores
                if ((v & 1) && variant_rg(MP, v) == variant_rg(MP, v & 2)) continue;
                for (int per : {1, 2, 4})
                    for (int gpc : {2, 4, 8, 16}) {
                        if (rc != STC_OK) break;
                        bt->tile[g][c] = BatchTile{true, v, per, gpc};
                        double ms = INFINITY;
                        rc = timed(&ms);
                        if (rc == STC_OK && ms < best_c) {
                            best_c = ms;
                            best = bt->tile[g][c];
                        }
                    }
            }
            bt->tile[g][c] = best;
            best_ms = best_c;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != STC_OK) return rc;
    // the members start again from e/N in their first stage, with the tuned
    // variants, under the caller's tolerance
    for (stc_handle *h : bt->members) {
        const int v0 = h->variant[0], v1 = h->variant[1];
        if ((rc = load_vector(h, nullptr, STC_MEM_HOST)) != STC_OK) return rc;
        h->variant[0] = v0;
        h->variant[1] = v1;
    }
    if ((rc = upload_lists(bt, bt->tol)) != STC_OK) return rc;
    if (ms_per_sweep) *ms_per_sweep = best_ms;
    return STC_OK;
}

stc_status stc_batch_get_tile(const stc_batch *bt, int32_t stage, int32_t mp, int32_t *variant,
                              int32_t *groups_per_item, int32_t *grid) {
    if (!bt || (stage != STC_FP64 && stage != STC_FP32) || mp > 128 || supported_mp(mp) != mp)
        return fail(STC_EINVAL, "need a batch, stage STC_FP64 or STC_FP32 and mp in 8, 16, 32, "
                                "64, 128");
    const int g = stage == STC_FP32 ? 1 : 0, c = class_of(mp);
    if (variant) *variant = tile_variant(bt, g, c);
    if (groups_per_item) *groups_per_item = bt->tile[g][c].per_item;
    if (grid) *grid = bt->tile[g][c].grid_per_cu * bt->cus;
    return STC_OK;
}

stc_status stc_batch_sweeps(stc_batch *bt, int64_t nsweeps, int32_t use_graph) {
    if (!bt || nsweeps < 0 || nsweeps > INT32_MAX) return fail(STC_EINVAL, "bad argument");
    if (nsweeps == 0) return STC_OK;
    if (!use_graph) {
        HIP_TRY(enqueue_batch(bt, nsweeps));
        return STC_OK;
    }
    const int groups = batch_shape(bt);
    if (!bt->exec || bt->graph_n != nsweeps || bt->graph_groups != groups) {
        drop_graph(bt);
        HIP_TRY(hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_batch(bt, nsweeps);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(bt->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(STC_EDEVICE, "graph capture: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        bt->graph = g;
        HIP_TRY(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
        bt->graph_n = nsweeps;
        bt->graph_groups = groups;
    }
    HIP_TRY(hipGraphLaunch(bt->exec, bt->stream));
    return STC_OK;
}

stc_status stc_batch_query(stc_batch *bt, int64_t *sweeps, int32_t *stopped, double *diff_1,
                           int32_t *status) {
    if (!bt) return fail(STC_EINVAL, "null batch");
    const int n = (int)bt->members.size();
    if (n == 0) return STC_OK;
    std::vector<QueryRow> rows(n);
    HIP_TRY(launch_batch_query(bt->d_states, n, bt->d_query, bt->stream));
    HIP_TRY(hipMemcpyAsync(rows.data(), bt->d_query, sizeof(QueryRow) * n, hipMemcpyDeviceToHost,
                           bt->stream));
    HIP_TRY(hipStreamSynchronize(bt->stream));
    for (int c = 0; c < n; ++c) {
        bt->members[c]->s = rows[c].last_sweep;
        if (sweeps) sweeps[c] = rows[c].sweeps;
        if (stopped) stopped[c] = rows[c].stopped;
        if (diff_1) diff_1[c] = rows[c].diff;
        if (status) status[c] = rows[c].status == kDevDegenerate ? STC_EDEGENERATE : STC_OK;
    }
    return STC_OK;
}

stc_status stc_batch_sync(stc_batch *bt) {
    if (!bt) return fail(STC_EINVAL, "null batch");
    HIP_TRY(hipStreamSynchronize(bt->stream));
    return STC_OK;
}

void stc_batch_destroy(stc_batch *bt) {
    if (!bt) return;
    drop_graph(bt);
    free_branches(bt);
    if (bt->own_stream) {
        (void)hipStreamSynchronize(bt->stream);
        (void)hipStreamDestroy(bt->stream);
    }
    delete bt;
}

}  // extern "C"
