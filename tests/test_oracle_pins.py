"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names the fact it uses: a closed form, a worked example printed in
the paper, a brute-force solve, a planted solution, or a spectral identity
stated in section 2.
"""
import os

import numpy as np
import pytest

import synth
from oracle import dense, gth, level_reduction, splittings, staircase


# --------------------------------------------------------------------------
# closed form: scalar birth-death chain, pi_i proportional to prod lam/mu
# --------------------------------------------------------------------------
def _bd_closed_form(lam, mu):
    L = lam.size
    w = np.ones(L)
    for i in range(1, L):
        w[i] = w[i - 1] * lam[i - 1] / mu[i]
    return w / w.sum()


@pytest.mark.parametrize("L,seed", [(12, 1), (40, 2), (7, 3)])
def test_birth_death_closed_form_gth_and_level_reduction(L, seed):
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.2, 2.0, L)
    mu = rng.uniform(0.2, 2.0, L)
    g = synth.birth_death(lam, mu)
    ref = _bd_closed_form(lam, mu)
    Q = dense.assemble_Q(g.blocks, g.sizes, g.b)
    assert np.abs(gth.gth(Q) - ref).sum() < 1e-14
    assert np.abs(level_reduction.level_reduction(g.blocks, g.sizes, g.b) - ref).sum() < 1e-14


@pytest.mark.parametrize("stair_type", [1, 2])
def test_birth_death_closed_form_staircase(stair_type):
    rng = np.random.default_rng(5)
    L = 24
    lam = rng.uniform(0.3, 1.0, L)
    mu = rng.uniform(0.6, 1.5, L)
    g = synth.birth_death(lam, mu)
    ref = _bd_closed_form(lam, mu)
    r = staircase.staircase_solve(g.blocks, g.sizes, g.b, stair_type=stair_type,
                                  tol=1e-15, maxit=20000)
    assert np.abs(r.x - ref).sum() < 1e-12


def test_residual_birth_death_closed_form():
    """(Q^T x)_i = lam_{i-1} x_{i-1} + mu_{i+1} x_{i+1} - (lam_i + mu_i) x_i."""
    rng = np.random.default_rng(9)
    L = 17
    lam = rng.uniform(0.2, 2.0, L)
    mu = rng.uniform(0.2, 2.0, L)
    lam[-1] = 0.0
    mu[0] = 0.0
    g = synth.birth_death(lam, mu)
    x = rng.random(L)
    want = -(lam + mu) * x
    want[1:] += lam[:-1] * x[:-1]
    want[:-1] += mu[1:] * x[1:]
    got = dense.residual_1(g.blocks, g.sizes, g.b, x)
    assert abs(got - np.abs(want).sum()) < 1e-13


# --------------------------------------------------------------------------
# brute force on tiny chains (a replaced-equation linear solve)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,m,last,seed", [(6, 3, None, 11), (5, 4, 2, 12), (9, 2, 1, 13)])
def test_gth_vs_bruteforce(L, m, last, seed):
    g = synth.qbd(L, m, seed, last=last)
    Q = dense.assemble_Q(g.blocks, g.sizes, g.b)
    ref = dense.nullspace_solve(Q)
    # independent second route: SVD null vector of Q^T
    _, _, vt = np.linalg.svd(Q.T)
    v = np.abs(vt[-1])
    v /= v.sum()
    assert np.abs(ref - v).sum() < 1e-12
    assert np.abs(gth.gth(Q) - ref).sum() < 1e-13


def test_gth_rejects_reducible():
    Q = np.array([[-1.0, 1.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    with pytest.raises(ValueError):
        gth.gth(Q)


# --------------------------------------------------------------------------
# planted stationary vector (detailed balance)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,m,b,last,seed", [(10, 4, 1, None, 21), (9, 5, 1, 3, 22),
                                             (12, 3, 2, None, 23), (11, 4, 2, 1, 24),
                                             (13, 3, 3, 2, 25), (14, 3, 4, None, 26)])
def test_planted_gth_and_level_reduction(L, m, b, last, seed):
    g, pstar = synth.planted_reversible(L, m, seed, b=b, last=last)
    Q = dense.assemble_Q(g.blocks, g.sizes, g.b)
    assert np.abs(gth.gth(Q) - pstar).sum() < 1e-13
    assert np.abs(level_reduction.level_reduction(g.blocks, g.sizes, g.b) - pstar).sum() < 1e-13
    assert dense.residual_1(g.blocks, g.sizes, g.b, pstar) < 1e-13


@pytest.mark.parametrize("b,stair_type", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (4, 2)])
def test_planted_staircase_converges(b, stair_type):
    g, pstar = synth.planted_reversible(8, 4, 31 + b, b=b)
    r = staircase.staircase_solve(g.blocks, g.sizes, g.b, stair_type=stair_type,
                                  tol=1e-15, maxit=50000)
    assert np.abs(r.x - pstar).sum() < 1e-12


def test_gth_equals_level_reduction_small_config_shape():
    """The two reference routes agree on the 64-level, m=16 QBD workload."""
    g = synth.qbd(64, 16, synth.config_seed(0))
    Q = dense.assemble_Q(g.blocks, g.sizes, g.b)
    p1 = gth.gth(Q)
    p2 = level_reduction.level_reduction(g.blocks, g.sizes, g.b)
    assert np.abs(p1 - p2).sum() < 1e-13
    assert np.all(p1 > 0) and abs(p1.sum() - 1) < 1e-15
    assert dense.residual_1(g.blocks, g.sizes, g.b, p1) < 1e-13


# --------------------------------------------------------------------------
# the paper's worked examples (Example 1 and Example 2, section 2)
# --------------------------------------------------------------------------
def _load_example(golden_dir):
    rows, spectra = [], {}
    with open(os.path.join(golden_dir, "example1.txt")) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert lines[0] == ["matrix"]
    for k in range(1, 5):
        rows.append([float(v) for v in lines[k]])
    for ln in lines[5:]:
        spectra[ln[0]] = np.array([float(v) for v in ln[1:]])
    return np.array(rows), spectra


def test_example_spectra(golden_dir):
    A, spectra = _load_example(golden_dir)
    for kind, want in spectra.items():
        got = splittings.spectrum(A, [1, 1, 1, 1], kind)
        assert np.allclose(np.sort(got.real), np.sort(want), atol=1e-12), kind
        assert np.allclose(got.imag, 0, atol=1e-12)


def test_example_jacobi_does_not_converge(golden_dir):
    """Example 1: with eigenvalue -1 the normalised Jacobi iteration cycles."""
    A, _ = _load_example(golden_dir)
    T = splittings.iteration_matrix(A, [1] * 4, "jacobi")
    x = np.array([0.4, 0.3, 0.2, 0.1])
    xs = []
    for _ in range(200):
        x = T @ x
        x = x / x.sum()
        xs.append(x)
    assert np.abs(xs[-1] - xs[-3]).sum() < 1e-12      # period 2
    assert np.abs(xs[-1] - xs[-2]).sum() > 1e-3       # but no fixed point


def test_example_stair_sweep_spectrum_matches_gs(golden_dir):
    """Example 2 via the sweep itself: the oracle sweep's linear map on the
    4-state example has the Gauss-Seidel spectrum {1, 1/4, 0, 0}."""
    A, spectra = _load_example(golden_dir)
    Q = A.T   # the sweep takes generator blocks: Q_{k,i} = A_{i,k}^T
    blocks = np.zeros((4, 3, 1, 1))
    for i in range(4):
        for d in (-1, 0, 1):
            if 0 <= i + d < 4:
                blocks[i, d + 1, 0, 0] = Q[i, i + d]
    sys = staircase.BlockSystem(blocks, [1, 1, 1, 1], 1)
    probe = np.array([0.1, 0.2, 0.3, 0.4])
    # the normalised map fixes the stationary vector and contracts by 1/4
    pi = dense.nullspace_solve(Q)
    zpi, _ = staircase.staircase_sweep(sys, pi, 1)
    assert np.abs(zpi - pi).sum() < 1e-14
    x = probe.copy()
    diffs = []
    for _ in range(16):
        x, d = staircase.staircase_sweep(sys, x, 1)
        diffs.append(d)
    ratios = np.array(diffs[9:]) / np.array(diffs[8:-1])
    assert np.allclose(ratios, 0.25, atol=1e-6)
    assert spectra["stair1"][1] == 0.25


# --------------------------------------------------------------------------
# spectral identity of section 2: block tridiagonal => BS and BGS share eigenvalues
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,m,last,seed", [(8, 4, None, 41), (7, 3, 2, 42), (10, 2, 1, 43)])
def test_stair_spectrum_equals_block_gauss_seidel(L, m, last, seed):
    """Eigenvalues well above the rounding floor agree (the zero eigenvalues
    of these defective iteration matrices come out of LAPACK as ~1e-5 noise).
    A third route pins both: on a two-cyclic block tridiagonal matrix the
    block Gauss-Seidel eigenvalues are the squares of the block Jacobi ones."""
    g = synth.qbd(L, m, seed, last=last)
    A = dense.assemble_A(g.blocks, g.sizes, g.b)
    gs = splittings.spectrum(A, g.sizes, "gs")
    jac = splittings.spectrum(A, g.sizes, "jacobi")
    floor = 1e-3
    gs_big = np.sort(np.abs(gs[np.abs(gs) > floor]))
    jac_sq = np.sort(np.abs(jac) ** 2)[::2]          # each mu^2 appears for +-mu
    jac_sq = jac_sq[jac_sq > floor]
    assert gs_big.size == jac_sq.size
    assert np.allclose(gs_big, jac_sq, rtol=1e-6)
    for kind in ("stair1", "stair2"):
        st = splittings.spectrum(A, g.sizes, kind)
        st_big = np.sort(np.abs(st[np.abs(st) > floor]))
        assert st_big.size == gs_big.size, kind
        assert np.allclose(st_big, gs_big, rtol=1e-6), kind
        assert abs(splittings.second_modulus(st) - splittings.second_modulus(gs)) < 1e-10


def test_jacobi_on_qbd_has_minus_one():
    """Block tridiagonal (two-cyclic) Q^T: block Jacobi has |lambda| = 1 twice,
    the failure mode shown by Example 1."""
    g = synth.qbd(8, 3, 44)
    A = dense.assemble_A(g.blocks, g.sizes, g.b)
    ev = splittings.spectrum(A, g.sizes, "jacobi")
    assert np.sum(np.abs(np.abs(ev) - 1.0) < 1e-9) == 2
    assert np.min(np.abs(ev + 1.0)) < 1e-9


# --------------------------------------------------------------------------
# the sweep: dense formula, fixed point, contraction rate
# --------------------------------------------------------------------------
@pytest.mark.parametrize("b,stair_type,last", [(1, 1, None), (1, 2, 2), (2, 1, None), (2, 2, 1),
                                               (3, 1, 2), (4, 2, None)])
def test_sweep_equals_dense_splitting(b, stair_type, last):
    """One sweep of Algorithm 2 = normalised M^{-1} N x with M the stair matrix
    (for b >= 2 the first loop gathers old values from every level of the
    band outside J_i)."""
    if b == 1:
        g = synth.qbd(9, 4, 50 + stair_type, last=last)
    elif b == 2:
        g = synth.banded(9, 4, 52 + stair_type, b=2, density=0.5, last=last)
    else:
        g = synth.skip_free(11, 4, 54 + b, b=b, last=last)
    A = dense.assemble_A(g.blocks, g.sizes, g.b)
    T = splittings.iteration_matrix(A, g.sizes, f"stair{stair_type}")
    x = synth.positive_start(g, 7)
    want = T @ x
    want /= want.sum()
    sys = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    z, err = staircase.staircase_sweep(sys, x, stair_type)
    assert np.abs(z - want).sum() < 1e-14
    assert abs(err - np.abs(want - x).sum()) < 1e-14


def test_jgs_sweep_equals_dense_splitting():
    g = synth.qbd(10, 3, 60, last=2)
    A = dense.assemble_A(g.blocks, g.sizes, g.b)
    chunks = [(0, 4), (4, 3), (7, 3)]
    T = splittings.iteration_matrix(A, g.sizes, "jgs", chunks)
    x = synth.positive_start(g, 8)
    want = T @ x
    want /= want.sum()
    z, _ = staircase.jgs_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x, chunks)
    assert np.abs(z - want).sum() < 1e-14


@pytest.mark.parametrize("stair_type", [1, 2])
def test_sweep_fixed_point(stair_type):
    g = synth.qbd(16, 8, 70, last=5)
    Q = dense.assemble_Q(g.blocks, g.sizes, g.b)
    pi = gth.gth(Q)
    z, err = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), pi,
                                       stair_type)
    assert err < 1e-14


def test_literal_J_reading_fails():
    """Reading guard: summing over k not in J_i with k = i included makes pi
    no longer a fixed point, so that reading cannot be the method."""
    g = synth.qbd(16, 8, 71)
    pi = gth.gth(dense.assemble_Q(g.blocks, g.sizes, g.b))
    sys = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    z, _ = staircase.staircase_sweep(sys, pi, 1, literal_J=True)
    assert np.abs(z - pi).sum() > 1e-2


def test_observed_contraction_matches_gamma():
    g = synth.qbd(8, 4, 72)
    A = dense.assemble_A(g.blocks, g.sizes, g.b)
    gamma = splittings.second_modulus(splittings.spectrum(A, g.sizes, "stair1"))
    r = staircase.staircase_solve(g.blocks, g.sizes, g.b, tol=1e-13, maxit=5000,
                                  keep_history=True)
    h = np.array(r.history)
    k0, k1 = len(h) // 2, len(h) - 2
    rate = (h[k1] / h[k0]) ** (1.0 / (k1 - k0))
    assert abs(rate - gamma) < 2e-3 * gamma


def test_degenerate_start_raises():
    """A start supported only on phase-A levels of a QBD maps to z = 0."""
    g = synth.qbd(6, 3, 73)
    x = np.zeros(g.N)
    x[: g.sizes[0]] = 1.0 / g.sizes[0]     # level 0: a phase-A level of type 1
    with pytest.raises(staircase.DegenerateIterate):
        staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x, 1)


def test_stop_rules_and_maxit():
    g = synth.qbd(12, 4, 74)
    r = staircase.staircase_solve(g.blocks, g.sizes, g.b, tol=1e-30, maxit=17)
    assert r.iters == 17 and not r.converged
    r = staircase.staircase_solve(g.blocks, g.sizes, g.b, tol=1e-12, maxit=10000,
                                  stop=staircase.STOP_RESIDUAL)
    assert r.converged and r.residual <= 1e-12


# --------------------------------------------------------------------------
# skip-free (M/G/1-type) generators with wide bands
# --------------------------------------------------------------------------
@pytest.mark.parametrize("b", [3, 4])
def test_skip_free_direct_solvers_agree_and_staircase_converges(b):
    """Level reduction (super-levels of b levels) equals dense GTH on a
    generator whose blocks below the first subdiagonal are zero, and the
    staircase iteration converges to it."""
    g = synth.skip_free(17, 4, 60 + b, b=b, last=3)
    assert not g.blocks[:, : b - 1].any()          # skip-free to the left
    Q = dense.assemble_Q(g.blocks, g.sizes, g.b)
    ref = gth.gth(Q)
    assert np.abs(level_reduction.level_reduction(g.blocks, g.sizes, g.b) - ref).sum() < 1e-13
    r = staircase.staircase_solve(g.blocks, g.sizes, g.b, tol=1e-15, maxit=50000)
    assert np.abs(r.x - ref).sum() < 1e-12
