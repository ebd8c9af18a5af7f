"""Pins of the oracle's staircase-preconditioned GMRES (CPU only).

  * the unnormalised operator T = M^{-1} N applied by the three loops of
    Algorithm 2 equals the dense stair-matrix formula on signed vectors;
  * the solve converges to the GTH vector (a direct solver);
  * GMRES with a restart longer than N reaches the null vector in one cycle
    (the Krylov space is then all of R^N), and its least-squares residual
    estimates never rise inside a cycle (the minimal-residual property);
  * a planted sign slip in the cycle's first residual makes it fail;
  * without drift it needs far fewer applications than sweeps.
The oracle is plain restarted GMRES; the product's rule for rejecting
stalled cycles is tested on the GPU as product behaviour.
"""
import numpy as np
import pytest

import synth
from oracle import dense, gth, krylov, splittings, staircase


def _banded():
    return synth.banded(24, 8, 5, b=2, density=0.4, last=5)


@pytest.mark.parametrize("stair_type", [1, 2])
def test_stair_apply_is_the_dense_operator(stair_type):
    g = _banded()
    A = dense.assemble_A(g.blocks, g.sizes, g.b)
    M = splittings.splitting_M(A, g.sizes, f"stair{stair_type}")
    v = np.random.default_rng(1).standard_normal(g.N)
    z = staircase.stair_apply(staircase.BlockSystem(g.blocks, g.sizes, g.b), v, stair_type)
    assert np.allclose(z, np.linalg.solve(M, (M - A) @ v), atol=1e-13, rtol=0)
    h = synth.localized(10, 6, 2, up=3, down=2, jumps=2, ragged=True)
    A = h.to_scipy().T.toarray()
    M = splittings.splitting_M(A, h.sizes, f"stair{stair_type}")
    v = np.random.default_rng(2).standard_normal(h.N)
    z = staircase.stair_apply(staircase.SparseBlockSystem(h.to_scipy(), h.sizes), v, stair_type)
    assert np.allclose(z, np.linalg.solve(M, (M - A) @ v), atol=1e-13, rtol=0)


@pytest.mark.parametrize("which", ["banded", "qbd", "general"])
def test_gmres_reaches_gth(which):
    if which == "general":
        g = synth.localized(12, 8, 9, up=3, down=2, jumps=2, ragged=True)
        sys = staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
        Q = g.to_scipy().toarray()
    else:
        g = _banded() if which == "banded" else synth.qbd(20, 8, 7, last=3)
        sys = staircase.BlockSystem(g.blocks, g.sizes, g.b)
        Q = dense.assemble_Q(g.blocks, g.sizes, g.b)
    r = krylov.gmres_solve(sys, restart=20, tol=1e-13, maxit=5000)
    assert r.converged
    assert np.abs(r.x - gth.gth(Q)).sum() < 1e-11


def test_full_gmres_converges_in_one_cycle_and_estimates_fall():
    g = synth.qbd(6, 4, 3, last=2)
    sys = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    x0 = np.full(g.N, 1.0 / g.N)
    x, applies, est = krylov.gmres_cycle(sys, x0, g.N + 1)
    assert sys.residual(x) < 1e-13
    # minimal residual: no rise while above the rounding floor
    floor = 1e-13 * est[0]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(est, est[1:]) if a > floor)
    assert min(est) < floor
    assert np.abs(x - gth.gth(dense.assemble_Q(g.blocks, g.sizes, g.b))).sum() < 1e-12


def test_sign_slip_in_the_first_residual_is_caught(monkeypatch):
    g = _banded()
    sys = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    real = staircase.stair_apply

    def flipped(sys_, x, stair_type=1, literal_J=False):
        # makes r = x - T x (= B x) instead of T x - x inside the cycle
        return 2.0 * x - real(sys_, x, stair_type, literal_J)
    calls = {"n": 0}

    def first_flipped(sys_, x, stair_type=1, literal_J=False):
        calls["n"] += 1
        return flipped(sys_, x, stair_type) if calls["n"] == 1 else real(sys_, x, stair_type)
    monkeypatch.setattr(krylov, "stair_apply", first_flipped)
    x, _, _ = krylov.gmres_cycle(sys, np.full(g.N, 1.0 / g.N), 20)
    pi = gth.gth(dense.assemble_Q(g.blocks, g.sizes, g.b))
    monkeypatch.setattr(krylov, "stair_apply", real)
    good, _, _ = krylov.gmres_cycle(sys, np.full(g.N, 1.0 / g.N), 20)
    assert np.abs(good - pi).sum() < 0.1 * np.abs(x - pi).sum()


def test_restarted_gmres_beats_the_stationary_sweeps_without_drift():
    """On a chain without drift restarted GMRES needs far fewer applications
    of T than the stationary iteration needs sweeps, and every cycle lowers
    the residual (the Krylov step of each cycle is the minimal-residual one)."""
    g = _banded()
    sys = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    stat = staircase.solve_system(sys, tol=1e-12, maxit=200_000, stop=staircase.STOP_RESIDUAL)
    r = krylov.gmres_solve(sys, restart=30, tol=1e-12, maxit=20_000)
    assert r.converged and r.applies * 5 < stat.iters
    assert all(b < a for a, b in zip(r.history, r.history[1:]))
