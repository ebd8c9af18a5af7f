"""Planted mistakes in the oracle (CPU only): each plausible slip must make
one of the pins fail.  The mutants are built here by patching oracle
functions for the duration of one test; the oracle itself is untouched."""
import numpy as np

import synth
from oracle import dense, gth, level_reduction, splittings, staircase


def _pi(g):
    return gth.gth(dense.assemble_Q(g.blocks, g.sizes, g.b))


def _fixed_point_error(g, stair_type=1):
    sys = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    z, _ = staircase.staircase_sweep(sys, _pi(g), stair_type)
    return np.abs(z - _pi(g)).sum()


def _dense_formula_error(g, stair_type=1):
    A = dense.assemble_A(g.blocks, g.sizes, g.b)
    T = splittings.iteration_matrix(A, g.sizes, f"stair{stair_type}")
    x = synth.positive_start(g, 3)
    want = T @ x
    want /= want.sum()
    z, _ = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x,
                                     stair_type)
    return np.abs(z - want).sum()


G = synth.qbd(10, 4, 99, last=3)


def test_unmutated_pins_hold():
    assert _fixed_point_error(G) < 1e-14
    assert _dense_formula_error(G) < 1e-14


def test_transposed_block_is_caught(monkeypatch):
    def wrong_A(self, i, k):   # uses Q_{i,k} instead of (Q_{k,i})^T
        d = k - i
        if abs(d) > self.b or not (0 <= k < self.L):
            return np.zeros((self.sizes[i], self.sizes[k]))
        return self.blocks[i, d + self.b, : self.sizes[i], : self.sizes[k]]
    monkeypatch.setattr(staircase.BlockSystem, "A", wrong_A)
    assert _fixed_point_error(G) > 1e-6


def test_swapped_phases_is_caught(monkeypatch):
    """Type 2 is a valid method too, so the fixed point cannot see this slip;
    the dense stair-matrix formula does."""
    real = staircase.phase_sets
    monkeypatch.setattr(staircase, "phase_sets", lambda L, t: real(L, 3 - t))
    assert _dense_formula_error(G) > 1e-6


def test_dropped_neighbour_is_caught(monkeypatch):
    """Moving one neighbour to the old-x side is still a regular splitting, so
    pi stays a fixed point; the stair-matrix formula catches it."""
    real = staircase.J_set

    def one_sided(i, L, t):
        J = real(i, L, t)
        return J[:1] if len(J) == 2 else J
    monkeypatch.setattr(staircase, "J_set", one_sided)
    assert _fixed_point_error(G) < 1e-13
    assert _dense_formula_error(G) > 1e-6


def test_gth_off_by_one_back_substitution_is_caught(monkeypatch):
    def bad_gth(Q):
        A = np.array(Q, dtype=np.float64, copy=True)
        N = A.shape[0]
        for k in range(N - 1, 0, -1):
            s = A[k, :k].sum()
            A[:k, k] /= s
            A[:k, :k] += np.outer(A[:k, k], A[k, :k])
        pi = np.zeros(N)
        pi[0] = 1.0
        for k in range(1, N):
            pi[k] = pi[:k - 1] @ A[:k - 1, k] if k > 1 else A[0, k]
        return pi / pi.sum()
    g = synth.qbd(5, 3, 98)
    ref = dense.nullspace_solve(dense.assemble_Q(g.blocks, g.sizes, g.b))
    assert np.abs(bad_gth(dense.assemble_Q(g.blocks, g.sizes, g.b)) - ref).sum() > 1e-6


def test_level_reduction_missing_update_is_caught(monkeypatch):
    real = level_reduction._super_levels

    def no_down(blocks, sizes, b):
        diag, up, down = real(blocks, sizes, b)
        return diag, up, [None if d is None else 0.5 * d for d in down]
    monkeypatch.setattr(level_reduction, "_super_levels", no_down)
    g, pstar = synth.planted_reversible(8, 3, 97)
    got = level_reduction.level_reduction(g.blocks, g.sizes, g.b)
    assert np.abs(got - pstar).sum() > 1e-6


def test_wrong_splitting_is_caught_by_example(golden_dir, monkeypatch):
    """A stair matrix built with the upper neighbour only would not give the
    printed Example 2 spectrum."""
    from test_oracle_pins import _load_example
    A, spectra = _load_example(golden_dir)
    real = splittings.splitting_M

    def upper_only(A_, sizes, kind_, chunks=None):
        M = real(A_, sizes, "jacobi")
        for i in range(M.shape[0] - 1):
            if (i + 1) % 2 == 0:
                M[i, i + 1] = A_[i, i + 1]
        return M
    monkeypatch.setattr(splittings, "splitting_M", upper_only)
    got = splittings.spectrum(A, [1] * 4, "stair1")
    assert not np.allclose(np.sort(got.real), np.sort(spectra["stair1"]), atol=1e-6)
