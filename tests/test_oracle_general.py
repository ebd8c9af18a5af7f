"""Pins of the oracle on generators of any block pattern (CPU only).

The sweep of Algorithm 2 on a SparseBlockSystem is pinned against facts that
do not come from that code:
  * the stair-matrix definition of section 2, built densely (splittings.py),
    gives the same normalised iterate M^{-1} N x;
  * GTH elimination (a textbook direct solver) gives the fixed point;
  * the mutual-exclusion model has a closed-form stationary vector: the
    processes are independent reversible two-state chains, and blocking the
    requests that would exceed r users truncates the joint chain to a subset
    of its states, which keeps the product form restricted to that subset
    (Kelly's truncation theorem for reversible chains).
Planted mistakes (a far block dropped, far levels read fresh) must fail them.
Algorithm 1 (JGS) on the same systems is pinned the same way: one sweep is
the normalised M^{-1} N x of the JGS splitting, whose M is written in the
test from the definition (block lower triangular inside each chunk), and the
GTH vector is its fixed point for every chunking.
"""
import numpy as np
import pytest

import synth
from oracle import gth, splittings, staircase


def _dense_step(g, x, stair_type):
    A = g.to_scipy().T.toarray()
    M = splittings.splitting_M(A, g.sizes, f"stair{stair_type}")
    z = np.linalg.solve(M, (M - A) @ x)
    return z / z.sum()


def _start(N, seed):
    x = np.random.default_rng(seed).uniform(0.5, 1.5, N)
    return x / x.sum()


def mutex_closed_form(g):
    return synth.mutual_exclusion_pi(g)


GENERAL = [
    dict(L=12, m=6, seed=1, up=2, down=2, jumps=2, ragged=True),
    dict(L=16, m=4, seed=2, up=16, down=1, jumps=0, ragged=False),   # block upper Hessenberg
    dict(L=10, m=8, seed=3, up=1, down=4, jumps=3, ragged=True),
    dict(L=2, m=5, seed=4, up=1, down=1, jumps=0, ragged=True),
    dict(L=9, m=1, seed=5, up=3, down=3, jumps=1, ragged=False),     # scalar levels
]


@pytest.mark.parametrize("cfg", GENERAL, ids=lambda c: f"L{c['L']}_m{c['m']}_s{c['seed']}")
@pytest.mark.parametrize("stair_type", [1, 2])
def test_general_sweep_equals_stair_matrix_definition(cfg, stair_type):
    g = synth.localized(**cfg)
    sys = staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
    x = _start(g.N, 7)
    z, err = staircase.staircase_sweep(sys, x, stair_type)
    want = _dense_step(g, x, stair_type)
    assert np.abs(z - want).sum() < 1e-13
    assert abs(err - np.abs(want - x).sum()) < 1e-13


@pytest.mark.parametrize("cfg", GENERAL[:3], ids=lambda c: f"L{c['L']}_m{c['m']}_s{c['seed']}")
def test_general_solve_reaches_gth(cfg):
    g = synth.localized(**cfg)
    pi = gth.gth(g.to_scipy().toarray())
    sys = staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
    z, _ = staircase.staircase_sweep(sys, pi, 1)
    assert np.abs(z - pi).sum() < 1e-13           # pi is a fixed point
    r = staircase.solve_system(sys, tol=1e-14, maxit=50_000, stop=staircase.STOP_RESIDUAL)
    assert r.converged
    assert np.abs(r.x - pi).sum() < 1e-9


def test_generator_shapes():
    g = synth.localized(16, 4, 2, up=16, down=1, jumps=0)
    Q = g.to_scipy().toarray()
    lev = g.level_of()
    r, c = np.nonzero(Q)
    assert (lev[c] - lev[r]).min() == -1          # block upper Hessenberg
    assert g.block_reach() == 15
    assert np.abs(Q.sum(axis=1)).max() < 1e-14
    assert (Q - np.diag(np.diag(Q)) >= 0).all()


def test_mutex_state_space_matches_the_model():
    g = synth.mutual_exclusion(16, 12, 0)
    assert g.N == 64839
    # the scalar bandwidth of this state order is the one the paper reports
    rows = np.repeat(np.arange(g.N), np.diff(g.indptr))
    assert int(np.abs(rows - g.indices).max()) == 13495
    assert np.abs(np.add.reduceat(g.data, g.indptr[:-1])).max() < 1e-13


@pytest.mark.parametrize("n,r,m", [(6, 3, 8), (8, 5, 16), (7, 7, 16)])
def test_mutex_closed_form_is_stationary_and_is_the_gth_vector(n, r, m):
    g = synth.mutual_exclusion(n, r, 11, m=m)
    pi = mutex_closed_form(g)
    assert np.abs(g.to_scipy().T @ pi).sum() < 1e-15
    assert np.abs(gth.gth(g.to_scipy().toarray()) - pi).sum() < 1e-13


@pytest.mark.parametrize("stair_type", [1, 2])
def test_mutex_oracle_solve_reaches_closed_form(stair_type):
    g = synth.mutual_exclusion(8, 5, 3, m=16)
    sys = staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
    r = staircase.solve_system(sys, stair_type=stair_type, tol=1e-14, maxit=20_000)
    assert r.converged
    assert np.abs(r.x - mutex_closed_form(g)).sum() < 1e-11


def test_banded_generator_gives_the_same_sweep_both_ways():
    g = synth.banded(14, 6, 5, b=2, density=0.4, last=4)
    import scipy.sparse as sp
    indptr, col, val = g.to_csr()
    Q = sp.csr_matrix((val, col, indptr), shape=(g.N, g.N))
    x = synth.positive_start(g, 2)
    za, _ = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x)
    zb, _ = staircase.staircase_sweep(staircase.SparseBlockSystem(Q, g.sizes), x)
    assert np.abs(za - zb).sum() < 1e-14


def test_general_residual_is_the_matrix_product():
    g = synth.localized(10, 5, 8, jumps=3, ragged=True)
    sys = staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
    x = _start(g.N, 1)
    want = np.abs(g.to_scipy().toarray().T @ x).sum()
    assert abs(sys.residual(x) - want) < 1e-14


# --- planted mistakes ------------------------------------------------------

def _jgs_chunks(L, p):
    return [(c * L // p, (c + 1) * L // p - c * L // p) for c in range(p)]


@pytest.mark.parametrize("cfg", GENERAL, ids=lambda c: f"L{c['L']}_m{c['m']}_s{c['seed']}")
def test_general_jgs_sweep_equals_dense_splitting(cfg):
    """Algorithm 1 on a SparseBlockSystem (the oracle of the GPU's
    any-pattern JGS): one sweep equals the normalised M^{-1} N x of the JGS
    splitting, with M written here from the method's definition: the blocks
    A_{i,k} with k <= i and i, k in one chunk (block lower triangular inside
    each chunk, nothing across).  At p = 1 that is block Gauss-Seidel's M and
    at p = L block Jacobi's, which the oracle's own splittings also give."""
    g = synth.localized(**cfg)
    A = g.to_scipy().T.toarray()
    lev = np.repeat(np.arange(g.L), g.sizes)
    sysg = staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
    x = _start(g.N, 11)
    for p in sorted({1, min(3, g.L), g.L}):
        chunks = _jgs_chunks(g.L, p)
        chunk_of = np.repeat(np.arange(p), [c for _, c in chunks])[lev]
        M = np.where((chunk_of[:, None] == chunk_of[None, :]) & (lev[:, None] >= lev[None, :]),
                     A, 0.0)
        assert np.array_equal(M, splittings.splitting_M(A, g.sizes, "jgs", chunks))
        if p == 1:
            assert np.array_equal(M, splittings.splitting_M(A, g.sizes, "gs"))
        if p == g.L:
            assert np.array_equal(M, splittings.splitting_M(A, g.sizes, "jacobi"))
        want = np.linalg.solve(M, (M - A) @ x)
        want /= want.sum()
        z, err = staircase.jgs_sweep(sysg, x, chunks)
        assert np.abs(z - want).sum() < 1e-13, p
        assert abs(err - np.abs(want - x).sum()) < 1e-13


def test_general_jgs_fixed_point_and_fresh_reads():
    """The GTH vector is a fixed point of every JGS sweep, and the chunks
    matter: on a generator with far jumps, p = 1 and p = L give different
    iterates from the same start (fresh against previous-iterate reads)."""
    g = synth.localized(12, 6, 1, up=2, down=2, jumps=3, ragged=True)
    pi = gth.gth(g.to_scipy().toarray())
    sysg = staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
    for p in (1, 4, 12):
        z, err = staircase.jgs_sweep(sysg, pi, _jgs_chunks(g.L, p))
        assert err < 1e-13 and np.abs(z - pi).sum() < 1e-13
    x = _start(g.N, 3)
    z1, _ = staircase.jgs_sweep(sysg, x, _jgs_chunks(g.L, 1))
    zL, _ = staircase.jgs_sweep(sysg, x, _jgs_chunks(g.L, g.L))
    assert np.abs(z1 - zL).sum() > 1e-3


def test_dropped_far_block_is_caught(monkeypatch):
    g = synth.localized(12, 6, 1, up=2, down=2, jumps=3, ragged=True)
    orig = staircase.SparseBlockSystem.band

    def near_only(self, i):   # forgets blocks more than one level away
        return [k for k in orig(self, i) if abs(k - i) <= 1]
    monkeypatch.setattr(staircase.SparseBlockSystem, "band", near_only)
    sys = staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
    x = _start(g.N, 7)
    z, _ = staircase.staircase_sweep(sys, x, 1)
    assert np.abs(z - _dense_step(g, x, 1)).sum() > 1e-6


def test_far_levels_read_fresh_is_caught(monkeypatch):
    """A sweep that also took the far levels from the fresh iterate (a block
    Gauss-Seidel slip) no longer matches the stair-matrix definition."""
    g = synth.localized(12, 6, 1, up=2, down=2, jumps=3, ragged=True)

    def fresh_far(i, L, stair_type):
        diag_only, stair = staircase.phase_sets(L, stair_type)
        if i in stair:
            return [k for k in range(L) if k != i and k in diag_only]
        return [i]
    monkeypatch.setattr(staircase, "J_set", fresh_far)
    sys = staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
    x = _start(g.N, 7)
    z, _ = staircase.staircase_sweep(sys, x, 1)
    assert np.abs(z - _dense_step(g, x, 1)).sum() > 1e-6


# --- Example 3 / Table 1 ---------------------------------------------------

def test_example3_matrix_profile():
    """n = 16 blocks of size k: block lower Hessenberg (one block column above
    the diagonal), scalar lower bandwidth 4k, a singular M-matrix whose
    columns sum to 0."""
    g = synth.hessenberg_mmatrix(16, 16, 0)
    A = g.to_scipy().T.toarray()
    off = A - np.diag(np.diag(A))
    i, j = np.nonzero(off)
    assert (i - j).max() == 64 and (j // 16 - i // 16).max() == 1
    assert off.min() >= 0.0 and np.abs(A.sum(axis=0)).max() < 1e-13


def test_example3_block_tridiagonal_partition_gives_bgs_spectrum():
    """With kp = 64 and k = 16 the partition makes A block tridiagonal, where
    section 2 proves block staircase and block Gauss-Seidel share their
    eigenvalues (Table 1 prints rho_2 = 1.0 there); block Jacobi has a second
    eigenvalue of modulus 1 (the printed rho_1 = inf)."""
    from oracle import table1
    g = synth.hessenberg_mmatrix(16, 16, 2)
    A = g.to_scipy().T.toarray()
    sizes = synth.equal_levels(g.N, 64)
    ev_gs = splittings.spectrum(A, sizes, "gs")
    ev_bs = splittings.spectrum(A, sizes, "stair1")
    big = np.abs(ev_gs) > 1e-6
    assert np.allclose(np.sort(np.abs(ev_gs[big])), np.sort(np.abs(ev_bs[np.abs(ev_bs) > 1e-6])),
                       atol=1e-10)
    gm = table1.gammas(A, sizes)
    r1, r2 = table1.ratios(gm)
    assert abs(r2 - 1.0) < 1e-8 and r1 == np.inf


def test_example3_staircase_close_to_gauss_seidel():
    """The qualitative claim of Example 3: at k = 64, kp = 16 the staircase
    spectral gap stays within a factor 2 of block Gauss-Seidel's (rho_2 in
    [1, 2]), while block Jacobi's is smaller still (rho_1 > 1)."""
    from oracle import table1
    g = synth.hessenberg_mmatrix(16, 64, 0)
    A = g.to_scipy().T.toarray()
    r1, r2 = table1.ratios(table1.gammas(A, synth.equal_levels(g.N, 16)))
    assert 1.0 < r1 < 2.0 and 1.0 <= r2 < 2.0


def test_band_stand_ins_have_the_paper_shapes():
    """The stand-ins for the second and third test matrices of section 3
    (small copies): generators inside the stated scalar band; the symmetric
    one has Q = Q^T, so its stationary vector is uniform, which GTH
    confirms; in levels of the stated size they are block tridiagonal
    (bandwidth below the level size) or reach two levels below and one above."""
    g = synth.banded_random(900, 40, 40, 1, symmetric=True, m=64)
    Q = g.to_scipy()
    assert abs(Q - Q.T).max() == 0.0
    assert np.abs(np.asarray(Q.sum(axis=1))).max() <= 1e-13
    r, c = Q.nonzero()
    assert np.abs(r - c).max() <= 40 and (Q.data[r != c] >= 0.0).all()
    assert g.block_reach() == 1
    pi = gth.gth(Q.toarray())
    assert np.abs(pi - 1.0 / g.N).max() <= 1e-13
    h = synth.banded_random(1000, 80, 50, 2, m=64)
    Q = h.to_scipy()
    r, c = Q.nonzero()
    assert (c - r).max() <= 50 and (r - c).max() <= 80
    lev = h.level_of()
    assert (lev[c] - lev[r]).max() == 1 and (lev[r] - lev[c]).max() == 2


def test_upper_hessenberg_stand_in_shape():
    """The stand-in for the first test matrix of section 3: in levels of k
    states, transitions go down at most one level and up any number of
    levels (block upper Hessenberg), and it is a generator."""
    k = 10
    g = synth.upper_hessenberg(600, k, 3, m=k)
    Q = g.to_scipy()
    assert np.abs(np.asarray(Q.sum(axis=1))).max() <= 1e-13
    r, c = Q.nonzero()
    assert (Q.data[r != c] >= 0.0).all()
    lr, lc = r // k, c // k
    assert (lr - lc).max() == 1 and (lc - lr).max() >= 3
    pi = gth.gth(Q.toarray())
    sys = staircase.SparseBlockSystem(Q, synth.equal_levels(g.N, 40))
    res = staircase.solve_system(sys, stair_type=1, tol=1e-13, maxit=50_000)
    assert np.abs(res.x - pi).sum() <= 1e-10


def test_large_partition_workloads_have_the_papers_sizes():
    """The large-partition bench builds its workloads at the sizes and
    partitions of section 3: N = 64839 (mutual exclusion), 110400 (first
    matrix, levels of 512), 91881 (second, levels of 2048, block
    tridiagonal as the paper notes), 79220 (third, levels of 512 to 2048);
    every one a generator (rows sum to 0, rates >= 0)."""
    import bench
    want_N = {"mutex": 64839, "uhess": 110400, "ncd": 91881, "prio": 79220}
    for name, build, _closed in bench.LARGE_BLOCK_WORKLOADS:
        g = build(synth.config_seed(3))
        m = int(name.rsplit("_m", 1)[1])
        assert g.N == want_N[name.split("_")[0]], name
        assert g.m == m and g.L == -(-g.N // m), name
        Q = g.to_scipy()
        assert np.abs(np.asarray(Q.sum(axis=1))).max() <= 1e-12, name
        r, c = Q.nonzero()
        assert (Q.data[r != c] >= 0.0).all(), name
        if name.startswith("ncd"):
            assert g.block_reach() == 1
