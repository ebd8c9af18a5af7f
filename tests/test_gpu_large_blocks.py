"""GPU parity for generators of any block pattern partitioned into large
levels (padded block sizes 512, 1024 and 2048: the partitions l = 512 to 2048
of the experiments in section 3).

These run the large-block kernels: per phase a gather launch (r_i into a
scratch vector) and an apply launch over column slices of W_i, one partial
slot per slice, and the MFMA inverse over many workgroups per level (64-wide
panels, the inverses stored tile-major).  The
oracle is the same SparseBlockSystem sweep as for the smaller blocks, on the
same seeded inputs.  Tolerances as for the other kernels: one FP64 sweep
agrees to 1e-13 in the 1-norm, one FP32 sweep to 1e-5; a converged FP64
vector agrees with the exact stationary vector to 1e-10.
"""
import numpy as np
import pytest

import synth
from oracle import staircase

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_07551_amd import stc
    stc.load_library()


def _say(msg):
    print(msg, flush=True)


def _solver(g, **kw):
    from paper_2302_07551_amd import Solver, stc
    kw.setdefault("format", "sparse")
    return Solver(None, g.sizes, stc.STC_ANY_PATTERN, csr=g.csr, **kw)


def _system(g):
    return staircase.SparseBlockSystem(g.to_scipy(), g.sizes)


def _start(g, seed):
    x = np.random.default_rng(seed).uniform(0.5, 1.5, g.N)
    return x / x.sum()


LARGE = [
    # 5 ragged levels of at most 512 (phase A: 3 levels, phase B: 2)
    ("loc_L5_m512_ragged", lambda: synth.localized(5, 512, 17, up=2, down=2, jumps=1, ragged=True,
                                                   density=0.004)),
    # block size 1000, padded to 1024
    ("loc_L4_m1000_ragged", lambda: synth.localized(4, 1000, 18, up=1, down=2, jumps=1,
                                                    ragged=True, density=0.002)),
    # 3797 states: one level of 2048 and a ragged one of 1749
    ("mutex_n12_r8_m2048", lambda: synth.mutual_exclusion(12, 8, 19, m=2048)),
    # 7099 states in 4 levels of 2048, the last of 955
    ("mutex_n13_r8_m2048", lambda: synth.mutual_exclusion(13, 8, 20, m=2048)),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("stair_type", [1, 2])
@pytest.mark.parametrize("name,make", LARGE, ids=[s[0] for s in LARGE])
def test_large_block_step_matches_oracle(name, make, stair_type, precision):
    g = make()
    _say(f"large-block step {name} type {stair_type} {precision}")
    x = _start(g, 31)
    zr, dr = staircase.staircase_sweep(_system(g), x, stair_type)
    s = _solver(g, precision=precision, stair_type=stair_type, poison=True)
    z, d = s.step(x)
    tol = 1e-13 if precision == "fp64" else 1e-5
    assert np.all(np.isfinite(z))
    assert np.abs(z - zr).sum() <= tol and abs(d - dr) <= tol
    s.close()


@pytest.mark.parametrize("stair_type", [1, 2])
@pytest.mark.parametrize("name,make", [LARGE[k] for k in (0, 3)],
                         ids=[LARGE[k][0] for k in (0, 3)])
def test_large_block_sweeps_on_the_resident_iterate(name, make, stair_type):
    """Bursts of sweeps (lagged normalisation, phase B's fold over the slice
    partials, the flush in the apply kernel's slices) follow the oracle's
    recurrence, and the changes are the oracle's, for both stair types."""
    g = make()
    _say(f"large-block sweeps {name} type {stair_type}")
    x = _start(g, 5)
    s = _solver(g, poison=True, stair_type=stair_type)
    s.load(x)
    diffs = s.sweeps(6, with_diffs=True)
    z = s.store()
    sys = _system(g)
    xr, want = x, []
    for _ in range(6):
        xr, dr = staircase.staircase_sweep(sys, xr, stair_type)
        want.append(dr)
    assert np.abs(z - xr).sum() <= 1e-13
    assert np.abs(np.asarray(diffs) - np.asarray(want[:-1])).max() <= 1e-13
    s.close()


def test_large_block_bursts_equal_single_sweeps():
    """One burst of 9 sweeps and 9 bursts of one sweep give the same iterate
    bit for bit (the flush's changes equal the next sweep's partials)."""
    g = LARGE[0][1]()
    x = _start(g, 8)
    a, b = _solver(g), _solver(g)
    a.load(x)
    a.sweeps(9)
    b.load(x)
    for _ in range(9):
        b.sweeps(1)
    assert np.array_equal(a.store(), b.store())
    a.close()
    b.close()


@pytest.mark.parametrize("k", [0, 1, 3])
def test_large_block_residual_matches_oracle(k):
    g = LARGE[k][1]()
    x = np.random.default_rng(3).standard_normal(g.N)
    s = _solver(g)
    r = s.residual(x)
    assert abs(r - _system(g).residual(x)) <= 1e-12 * max(1.0, r)
    s.close()


@pytest.mark.parametrize("stair_type", [1, 2])
def test_large_block_diff_stop_iteration_count(stair_type):
    g = synth.localized(5, 600, 22, up=2, down=1, jumps=1, ragged=True, density=0.003)
    _say(f"large-block iteration count type {stair_type}")
    want = staircase.solve_system(_system(g), stair_type=stair_type, tol=1e-10, maxit=20_000)
    s = _solver(g, stair_type=stair_type)
    pi, info = s.solve(tol=1e-10, maxit=20_000)
    assert abs(info["iters"] - want.iters) <= max(2, want.iters // 100)
    assert np.abs(pi - want.x).sum() <= 1e-9
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_large_block_mutex_solve_reaches_closed_form(precision):
    g = synth.mutual_exclusion(13, 8, 23, m=2048)
    _say(f"mutex n13 m2048 solve {precision}")
    s = _solver(g, precision=precision)
    pi, info = s.solve(tol=1e-13, maxit=100_000)
    assert info["status"] == 0
    assert np.abs(pi - synth.mutual_exclusion_pi(g)).sum() <= 1e-10
    if precision == "mixed":
        assert info["iters_fp32"] > 0
    s.close()


@pytest.mark.parametrize("m", [512, 1024, 2048])
def test_large_block_mutex_full_size_solve(m):
    """The mutual-exclusion model at the paper's size (N = 64839) in levels
    of 512, 1024 or 2048 states: the solve to 1e-13 reaches the closed-form
    stationary vector.  (The oracle's dense blocks of this partition would
    take tens of GB, so the full-size check is against the closed form.)"""
    g = synth.mutual_exclusion(16, 12, synth.config_seed(3), m=m)
    s = _solver(g)
    pi, info = s.solve(tol=1e-13, maxit=100_000)
    err = np.abs(pi - synth.mutual_exclusion_pi(g)).sum()
    _say(f"mutex full m={m}: iters {info['iters']} err {err:.2e} res {info['residual_1']:.2e}")
    assert info["status"] == 0 and err <= 1e-10
    s.close()


@pytest.mark.parametrize("m", [512, 2048])
def test_large_block_singular_diagonal_block(m):
    """A level whose states can never leave it makes Q_ii singular: setup
    reports STC_ESINGULAR (the pivot check of the panel inverses)."""
    from paper_2302_07551_amd import Solver, stc
    g = synth.localized(4, m, 24, up=1, down=1, jumps=0, backbone=0.0,
                        density=8.0 / m)
    Q = g.to_scipy().tolil()
    off = g.offsets
    lev = 2
    for r in range(off[lev], off[lev + 1]):
        for c in list(Q.rows[r]):
            if not (off[lev] <= c < off[lev + 1]):
                Q[r, c] = 0.0
    Q = Q.tocsr()
    Q.setdiag(0.0)
    Q.setdiag(-np.asarray(Q.sum(axis=1)).ravel())
    Q.eliminate_zeros()
    Q.sort_indices()
    with pytest.raises(stc.StcError) as e:
        Solver(None, g.sizes, stc.STC_ANY_PATTERN, csr=(Q.indptr, Q.indices, Q.data),
               format="sparse")
    assert e.value.status == stc.STC_ESINGULAR


def test_large_block_load_policies_agree():
    """Plain and non-temporal loads (the kernels' one variant bit) give
    bitwise the same sweeps."""
    from paper_2302_07551_amd import stc
    g = LARGE[1][1]()
    x = _start(g, 2)
    a, b = _solver(g), _solver(g)
    stc.stc_set_variant(a.h, stc.STC_FP64, 0)
    stc.stc_set_variant(b.h, stc.STC_FP64, 2)
    for s in (a, b):
        s.load(x)
        s.sweeps(5)
    assert np.array_equal(a.store(), b.store())
    a.close()
    b.close()


FULL_SIZE = [
    ("mutex_n16_r12_m512", lambda sd: synth.mutual_exclusion(16, 12, sd, m=512)),
    ("prio_N79220_m1024", lambda sd: synth.banded_random(79220, 2370, 1585, sd, m=1024)),
    ("ncd_N91881_bw1135_m2048",
     lambda sd: synth.banded_random(91881, 1135, 1135, sd, symmetric=True, m=2048)),
]


@pytest.mark.parametrize("name,make", FULL_SIZE, ids=[f[0] for f in FULL_SIZE])
def test_large_block_full_size_sweep_matches_c_oracle(name, make):
    """The large-partition workloads at their full sizes (N = 64839 to
    91881), as the benchmark builds them: one FP64 sweep under both load
    policies, element by element against the oracle's C/OpenMP sweep of the
    whole chain (LU-factored diagonal blocks), with no fitted scalar; and
    the change."""
    from oracle import csweep
    from paper_2302_07551_amd import stc
    g = make(synth.config_seed(3))
    x = _start(g, 12)
    c = csweep.CGenSweep(g.to_scipy(), g.sizes, stair_type=1)
    zr = np.zeros(g.N)
    dr = c.sweep(x, zr)
    s = _solver(g)
    for variant in (0, 2):
        stc.stc_set_variant(s.h, stc.STC_FP64, variant)
        z, d = s.step(x)
        err = np.abs(z - zr).sum()
        _say(f"full size {name} variant {variant}: |z - z_oracle|_1 = {err:.2e}")
        assert err <= 1e-13 and abs(d - dr) <= 1e-13
    s.close()
