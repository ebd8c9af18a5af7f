/*
 * Algorithm 2 (block staircase splitting) as plain C with OpenMP loops over
 * levels: the same three parallel loops and serial normalisation as the
 * algorithm in section 2, in FP64, with an LU (partial pivoting) solve per
 * diagonal block.  It mirrors the paper's own C++/OpenMP implementation
 * (section 3) and is used only to time a CPU baseline.
 *
 * TEST INFRASTRUCTURE ONLY: part of the oracle; shares no code with the HIP
 * library.
 *
 * Banded data: generator blocks blocks[i][d+b] = Q_{i,i+d}, each m x m row-major,
 * zero padded; vectors are padded [L][m].  The matrix the algorithm acts on is
 * A = Q^T, whose block A_{i,k} is (Q_{k,i})^T.  Same readings as the Python
 * oracle: the first loop skips k = i as well as J_i; err is measured after
 * normalisation.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#include <xmmintrin.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double *qblock(const double *blocks, int m, int b, int row_level, int d)
{
    return blocks + ((size_t)row_level * (2 * b + 1) + (size_t)(d + b)) * (size_t)m * m;
}

/* y += sign * A_{i,k} v  with A_{i,k}[r][c] = Q_{k,i}[c][r] */
static void gemv_Aik(const double *blocks, const int *sizes, int m, int b, int i, int k,
                     const double *v, double *y, double sign)
{
    const double *Q = qblock(blocks, m, b, k, i - k);
    int ni = sizes[i], nk = sizes[k];
    for (int c = 0; c < nk; ++c) {
        double vc = sign * v[c];
        const double *row = Q + (size_t)c * m;
        for (int r = 0; r < ni; ++r) y[r] += row[r] * vc;
    }
}

static int is_stair_row(int i, int stair_type)
{
    /* 0-based level i is 1-based row i+1; type 1: odd 1-based rows are diagonal-only */
    int diag_only_parity = (stair_type == 1) ? 0 : 1;
    return (i % 2) != diag_only_parity;
}

/* LU with partial pivoting of A_ii = Q_ii^T (n x n) into lu (m x m row-major). */
int cs_factor(int L, int m, int b, const int *sizes, const double *blocks,
              double *lu, int *piv)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int i = 0; i < L; ++i) {
        int n = sizes[i];
        double *a = lu + (size_t)i * m * m;
        int *p = piv + (size_t)i * m;
        const double *Q = qblock(blocks, m, b, i, 0);
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) a[(size_t)r * m + c] = Q[(size_t)c * m + r];
        for (int j = 0; j < n; ++j) {
            int best = j;
            for (int r = j + 1; r < n; ++r)
                if (fabs(a[(size_t)r * m + j]) > fabs(a[(size_t)best * m + j])) best = r;
            p[j] = best;
            if (best != j)
                for (int c = 0; c < n; ++c) {
                    double t = a[(size_t)j * m + c];
                    a[(size_t)j * m + c] = a[(size_t)best * m + c];
                    a[(size_t)best * m + c] = t;
                }
            double d = a[(size_t)j * m + j];
            if (d == 0.0) { bad += 1; break; }
            for (int r = j + 1; r < n; ++r) {
                double f = a[(size_t)r * m + j] / d;
                a[(size_t)r * m + j] = f;
                for (int c = j + 1; c < n; ++c) a[(size_t)r * m + c] -= f * a[(size_t)j * m + c];
            }
        }
    }
    return bad ? -1 : 0;
}

static void lu_solve(const double *a, const int *p, int n, int m, double *x)
{
    for (int j = 0; j < n; ++j) {
        if (p[j] != j) { double t = x[j]; x[j] = x[p[j]]; x[p[j]] = t; }
    }
    for (int r = 1; r < n; ++r) {
        double s = x[r];
        for (int c = 0; c < r; ++c) s -= a[(size_t)r * m + c] * x[c];
        x[r] = s;
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = x[r];
        for (int c = r + 1; c < n; ++c) s -= a[(size_t)r * m + c] * x[c];
        x[r] = s / a[(size_t)r * m + r];
    }
}

/* One sweep from the normalised padded iterate x into z; *err = ||z - x||_1.
 * Returns 0, or -1 if e^T z is not positive and finite. */
int cs_sweep(int L, int m, int b, const int *sizes, const double *blocks,
             const double *lu, const int *piv, int stair_type,
             const double *x, double *z, double *err)
{
    /* first loop: z_i = - sum_{k outside J_i and k != i} A_{i,k} x_k */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L; ++i) {
        double *zi = z + (size_t)i * m;
        memset(zi, 0, sizeof(double) * (size_t)m);
        int stair = is_stair_row(i, stair_type);
        for (int k = i - b; k <= i + b; ++k) {
            if (k < 0 || k >= L || k == i) continue;
            if (stair && (k == i - 1 || k == i + 1)) continue;
            gemv_Aik(blocks, sizes, m, b, i, k, x + (size_t)k * m, zi, -1.0);
        }
    }
    /* second loop: diagonal-only rows */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L; ++i) {
        if (is_stair_row(i, stair_type)) continue;
        lu_solve(lu + (size_t)i * m * m, piv + (size_t)i * m, sizes[i], m, z + (size_t)i * m);
    }
    /* third loop: stair rows from the fresh neighbours */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < L; ++i) {
        if (!is_stair_row(i, stair_type)) continue;
        double *zi = z + (size_t)i * m;
        for (int k = i - 1; k <= i + 1; k += 2) {
            if (k < 0 || k >= L) continue;
            gemv_Aik(blocks, sizes, m, b, i, k, z + (size_t)k * m, zi, -1.0);
        }
        lu_solve(lu + (size_t)i * m * m, piv + (size_t)i * m, sizes[i], m, zi);
    }
    /* normalisation and change, serial as in the algorithm */
    size_t n = (size_t)L * m;
    double s = 0.0;
    for (size_t j = 0; j < n; ++j) s += z[j];
    if (!(s > 0.0) || !isfinite(s)) return -1;
    double e = 0.0;
    for (size_t j = 0; j < n; ++j) {
        z[j] /= s;
        e += fabs(z[j] - x[j]);
    }
    *err = e;
    return 0;
}

/* ---------------------------------------------------------------------------
 * Generators of any block pattern (the general localized case of section 2).
 * The matrix the algorithm acts on, A = Q^T, is given directly as compact CSR
 * rows (row r of A = column r of Q), states numbered level by level with
 * offsets off[0..L]; vectors are compact, length N = off[L].
 * ------------------------------------------------------------------------- */

static int level_of(const long long *off, int L, long long c)
{
    int lo = 0, hi = L - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (off[mid] <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* LU with partial pivoting of each diagonal block A_ii (n_i x n_i, padded to
 * m x m in lu) taken from the CSR rows. */
int cs_gen_factor(int L, int m, const long long *off, const long long *rp, const int *col,
                  const double *val, double *lu, int *piv)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(+ : bad)
    for (int i = 0; i < L; ++i) {
        int n = (int)(off[i + 1] - off[i]);
        double *a = lu + (size_t)i * m * m;
        int *p = piv + (size_t)i * m;
        memset(a, 0, sizeof(double) * (size_t)m * m);
        for (int r = 0; r < n; ++r)
            for (long long q = rp[off[i] + r]; q < rp[off[i] + r + 1]; ++q) {
                long long c = col[q];
                if (c >= off[i] && c < off[i + 1]) a[(size_t)r * m + (c - off[i])] = val[q];
            }
        for (int j = 0; j < n; ++j) {
            int best = j;
            for (int r = j + 1; r < n; ++r)
                if (fabs(a[(size_t)r * m + j]) > fabs(a[(size_t)best * m + j])) best = r;
            p[j] = best;
            if (best != j)
                for (int c = 0; c < n; ++c) {
                    double t = a[(size_t)j * m + c];
                    a[(size_t)j * m + c] = a[(size_t)best * m + c];
                    a[(size_t)best * m + c] = t;
                }
            double d = a[(size_t)j * m + j];
            if (d == 0.0) { bad += 1; break; }
            for (int r = j + 1; r < n; ++r) {
                double f = a[(size_t)r * m + j] / d;
                a[(size_t)r * m + j] = f;
                for (int c = j + 1; c < n; ++c) a[(size_t)r * m + c] -= f * a[(size_t)j * m + c];
            }
        }
    }
    return bad ? -1 : 0;
}

/* One sweep of Algorithm 2 from the normalised compact iterate x into z. */
int cs_gen_sweep(int L, int m, const long long *off, const long long *rp, const int *col,
                 const double *val, const double *lu, const int *piv, int stair_type,
                 const double *x, double *z, double *err)
{
    /* first loop: z_i = - sum over the entries of A's rows of level i whose
     * column lies outside level i and, on a stair row, outside J_i */
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < L; ++i) {
        int stair = is_stair_row(i, stair_type);
        for (long long r = off[i]; r < off[i + 1]; ++r) {
            double s = 0.0;
            for (long long q = rp[r]; q < rp[r + 1]; ++q) {
                long long c = col[q];
                if (c >= off[i] && c < off[i + 1]) continue;
                if (stair) {
                    int k = level_of(off, L, c);
                    if (k == i - 1 || k == i + 1) continue;
                }
                s += val[q] * x[c];
            }
            z[r] = -s;
        }
    }
    /* second loop: diagonal-only rows */
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < L; ++i) {
        if (is_stair_row(i, stair_type)) continue;
        lu_solve(lu + (size_t)i * m * m, piv + (size_t)i * m, (int)(off[i + 1] - off[i]), m,
                 z + off[i]);
    }
    /* third loop: stair rows from the fresh values of levels i - 1, i + 1 */
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < L; ++i) {
        if (!is_stair_row(i, stair_type)) continue;
        for (long long r = off[i]; r < off[i + 1]; ++r) {
            double s = 0.0;
            for (long long q = rp[r]; q < rp[r + 1]; ++q) {
                long long c = col[q];
                if (c >= off[i] && c < off[i + 1]) continue;
                int k = level_of(off, L, c);
                if (k == i - 1 || k == i + 1) s += val[q] * z[c];
            }
            z[r] -= s;
        }
        lu_solve(lu + (size_t)i * m * m, piv + (size_t)i * m, (int)(off[i + 1] - off[i]), m,
                 z + off[i]);
    }
    /* normalisation and change, serial */
    long long n = off[L];
    double s = 0.0;
    for (long long j = 0; j < n; ++j) s += z[j];
    if (!(s > 0.0) || !isfinite(s)) return -1;
    double e = 0.0;
    for (long long j = 0; j < n; ++j) {
        z[j] /= s;
        e += fabs(z[j] - x[j]);
    }
    *err = e;
    return 0;
}

/* The calling thread's SSE control word (MXCSR): bit 15 flush-to-zero, bit 6
 * denormals-are-zero.  The sweeps use the compiler's defaults (neither set),
 * so subnormal iterate entries are computed in full. */
unsigned cs_mxcsr(void)
{
    return _mm_getcsr();
}

int cs_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}
