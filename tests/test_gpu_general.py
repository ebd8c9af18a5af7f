"""GPU parity for generators of any block pattern (b = STC_ANY_PATTERN).

The HIP path (per-level near / far ELL with 32-bit gather indices) against
the oracle's SparseBlockSystem sweep on the same seeded inputs, and converged
vectors against the closed-form stationary vector of the mutual-exclusion
model.  Tolerances as for the banded kernels: one FP64 sweep agrees to 1e-13
in the 1-norm, one FP32 sweep to 1e-5; converged FP64 vectors agree with the
exact stationary vector to 1e-10 (change stop 1e-13).
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


def mutex_closed_form(g):
    return synth.mutual_exclusion_pi(g)


GENERAL = [
    ("loc_L12_m6_ragged", lambda: synth.localized(12, 6, 1, up=2, down=2, jumps=2, ragged=True)),
    ("hess_L16_m8", lambda: synth.localized(16, 8, 2, up=16, down=1, jumps=0)),
    ("loc_L10_m32_ragged", lambda: synth.localized(10, 32, 3, up=1, down=4, jumps=3, ragged=True)),
    ("loc_L2_m5", lambda: synth.localized(2, 5, 4, ragged=True)),
    ("loc_L3_m4", lambda: synth.localized(3, 4, 14, up=2, down=2)),
    ("loc_L9_m1", lambda: synth.localized(9, 1, 5, up=3, down=3, jumps=1)),
    ("loc_L21_m64_ragged", lambda: synth.localized(21, 64, 6, up=3, down=3, jumps=2, ragged=True,
                                                   density=0.05)),
    ("loc_L7_m128", lambda: synth.localized(7, 128, 7, up=2, down=6, jumps=1, density=0.03)),
    ("mutex_n8_r5_m16", lambda: synth.mutual_exclusion(8, 5, 3, m=16)),
    ("mutex_n10_r6_m32", lambda: synth.mutual_exclusion(10, 6, 4, m=32)),
    # blocks of 256 (the paper's own partition size for this model)
    ("loc_L5_m256_ragged", lambda: synth.localized(5, 256, 15, up=2, down=2, jumps=1,
                                                   ragged=True, density=0.02)),
    ("mutex_n11_r7_m256", lambda: synth.mutual_exclusion(11, 7, 16, m=256)),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("stair_type", [1, 2])
@pytest.mark.parametrize("name,make", GENERAL, ids=[s[0] for s in GENERAL])
def test_general_step_matches_oracle(name, make, stair_type, precision):
    g = make()
    _say(f"general step {name} type {stair_type} {precision}")
    x = _start(g, 31)
    zr, dr = staircase.staircase_sweep(_system(g), x, stair_type)
    s = _solver(g, precision=precision, stair_type=stair_type, poison=True)
    z, d = s.step(x)
    tol = 1e-13 if precision == "fp64" else 1e-5
    assert np.all(np.isfinite(z))
    assert np.abs(z - zr).sum() <= tol and abs(d - dr) <= tol
    assert np.isfinite(s.residual(x))
    s.close()


@pytest.mark.parametrize("name,make", [GENERAL[k] for k in (0, 1, 6, 9)],
                         ids=[GENERAL[k][0] for k in (0, 1, 6, 9)])
def test_general_sweeps_on_the_resident_iterate(name, make):
    """Bursts of sweeps (lagged normalisation, phase B's fold, the flush)
    follow the oracle's recurrence, and the changes are the oracle's."""
    g = make()
    _say(f"general sweeps {name}")
    x = _start(g, 5)
    s = _solver(g, poison=True)
    s.load(x)
    diffs = s.sweeps(6, with_diffs=True)
    z = s.store()
    sys = _system(g)
    xr, want = x, []
    for _ in range(6):
        xr, dr = staircase.staircase_sweep(sys, xr, 1)
        want.append(dr)
    assert np.abs(z - xr).sum() <= 1e-13
    # the changes of sweeps 1 .. n-1 (the last one is read with the iterate)
    assert np.abs(np.asarray(diffs) - np.asarray(want[:-1])).max() <= 1e-13
    s.close()


def test_general_residual_matches_oracle():
    g = synth.localized(14, 16, 8, up=2, down=3, jumps=3, ragged=True)
    x = np.random.default_rng(3).standard_normal(g.N)
    s = _solver(g)
    r = s.residual(x)
    assert abs(r - _system(g).residual(x)) <= 1e-12 * max(1.0, r)
    s.close()


@pytest.mark.parametrize("stair_type", [1, 2])
def test_general_diff_stop_iteration_count(stair_type):
    g = synth.localized(12, 8, 9, up=3, down=2, jumps=2, ragged=True)
    _say(f"general iteration count type {stair_type}")
    want = staircase.solve_system(_system(g), stair_type=stair_type, tol=1e-10, maxit=20_000)
    s = _solver(g, stair_type=stair_type)
    pi, info = s.solve(tol=1e-10, maxit=20_000)
    assert abs(info["iters"] - want.iters) <= max(2, want.iters // 100)
    assert np.abs(pi - want.x).sum() <= 1e-9
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mutex_solve_reaches_closed_form(precision):
    g = synth.mutual_exclusion(10, 6, 4, m=32)
    _say(f"mutex n10 solve {precision}")
    s = _solver(g, precision=precision)
    pi, info = s.solve(tol=1e-13, maxit=100_000)
    assert info["status"] == 0
    assert np.abs(pi - mutex_closed_form(g)).sum() <= 1e-10
    if precision == "mixed":
        assert info["iters_fp32"] > 0
    s.close()


def test_general_deterministic_and_profiled():
    from paper_2302_07551_amd import stc
    g = synth.localized(30, 16, 10, up=3, down=3, jumps=2)
    a, b = _solver(g), _solver(g)
    p1, i1 = a.solve(tol=1e-12, maxit=20_000)
    p2, i2 = a.solve(tol=1e-12, maxit=20_000)
    assert i1["iters"] == i2["iters"] and np.array_equal(p1, p2)
    a.load(None)
    b.load(None)
    a.sweeps(7)
    ms_a, ms_b, ms_f, ms_s = stc.stc_profile_sweeps(b.h, 7)
    assert np.array_equal(a.store(), b.store())
    assert ms_a > 0 and ms_b > 0 and ms_a + ms_b <= ms_s * 1.001 + 1e-3
    ba, bb = stc.stc_phase_bytes(a.h)
    assert ba > 0 and bb > 0
    a.close()
    b.close()


def test_banded_generator_any_pattern_equals_banded_path():
    """A pentadiagonal generator given as a pattern of any shape sweeps to the
    same iterate as the banded kernels (to rounding)."""
    from paper_2302_07551_amd import Solver, stc
    g = synth.banded(20, 32, 41, b=2, density=0.3, last=9)
    ip, ix, v = g.to_csr()
    x = synth.positive_start(g, 4)
    band = Solver(g.blocks, g.sizes, 2)
    anyp = Solver(None, g.sizes, stc.STC_ANY_PATTERN, csr=(ip, ix, v), format="sparse", m=g.m)
    za, da = band.step(x)
    zb, db = anyp.step(x)
    assert np.abs(za - zb).sum() <= 1e-13 and abs(da - db) <= 1e-13
    band.close()
    anyp.close()


def test_batch_rejects_any_pattern_chains():
    from paper_2302_07551_amd import Batch, stc
    g = synth.localized(8, 8, 12)
    s = _solver(g)
    bt = Batch(4, 64)
    with pytest.raises(stc.StcError) as e:
        bt.set([s], tol=0.0)
    assert e.value.status == stc.STC_EINVAL
    bt.close()
    s.close()


@pytest.mark.parametrize("m", [128, 256])
def test_mutex_full_size_step_and_solve(m):
    """The mutual-exclusion model at the paper's size (16 processes, at most
    12 users: N = 64839; 507 levels of 128 states, nonzero blocks up to 106
    levels from the diagonal, or the paper's own partition into 254 levels
    of 256), in the launch configuration the benchmark times: one sweep
    against the oracle, then a solve to the paper's change tolerance 1e-9
    and on to 1e-13, checked against the closed form."""
    g = synth.mutual_exclusion(16, 12, synth.config_seed(3), m=m)
    x = _start(g, 9)
    s = _solver(g)
    z, d = s.step(x)
    zr, dr = staircase.staircase_sweep(_system(g), x, 1)
    _say(f"mutex full step m={m}: |z-zr|_1 = {np.abs(z - zr).sum():.2e}")
    assert np.abs(z - zr).sum() <= 1e-13 and abs(d - dr) <= 1e-13
    exact = mutex_closed_form(g)
    pi, info = s.solve(tol=1e-9, maxit=10_000)
    _say(f"mutex full solve 1e-9: iters {info['iters']} err {np.abs(pi - exact).sum():.2e}")
    assert info["status"] == 0
    pi, info = s.solve(tol=1e-13, maxit=100_000)
    err = np.abs(pi - exact).sum()
    _say(f"mutex full solve 1e-13: iters {info['iters']} err {err:.2e} res {info['residual_1']:.2e}")
    assert info["status"] == 0 and err <= 1e-10
    s.close()


def test_load_policies_agree_and_default_by_size():
    """The kernel's one variant bit is its load policy (plain or non-temporal):
    both give bitwise the same sweeps.  Small stages default to plain loads
    (they stay in the last-level cache); a stage above 256 MB streams."""
    from paper_2302_07551_amd import stc
    g = synth.localized(24, 32, 15, up=3, down=2, jumps=2, ragged=True)
    x = _start(g, 2)
    a, b = _solver(g), _solver(g)
    assert stc.stc_get_variant(a.h, stc.STC_FP64) == 0
    stc.stc_set_variant(b.h, stc.STC_FP64, 2)
    for s in (a, b):
        s.load(x)
        s.sweeps(5)
    assert np.array_equal(a.store(), b.store())
    stc.stc_autotune(a.h, 3)
    assert stc.stc_get_variant(a.h, stc.STC_FP64) in (0, 2)
    a.close()
    b.close()
    big = synth.localized(2200, 128, 16, up=1, down=1, jumps=1, density=0.01)
    _say("large any-pattern chain: default load policy")
    s = _solver(big)
    assert stc.stc_get_variant(s.h, stc.STC_FP64) == 2   # 2200 x 128 KB of inverses
    x = _start(big, 3)
    s.load(x)
    s.sweeps(3)
    z_nt = s.store()
    stc.stc_set_variant(s.h, stc.STC_FP64, 0)
    s.load(x)
    s.sweeps(3)
    assert np.array_equal(z_nt, s.store())
    s.close()


@pytest.mark.parametrize("m", [8, 256])
def test_any_pattern_singular_diagonal_block(m):
    """A level whose states can never leave it makes Q_ii singular: setup
    reports STC_ESINGULAR (the inverse kernel's pivot check; at m = 256 the
    elimination in global memory)."""
    from paper_2302_07551_amd import stc
    g = synth.localized(6, m, 21, up=1, down=1, jumps=0, backbone=0.0)
    Q = g.to_scipy().tolil()
    off = g.offsets
    lev = 3
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
        from paper_2302_07551_amd import Solver
        Solver(None, g.sizes, stc.STC_ANY_PATTERN, csr=(Q.indptr, Q.indices, Q.data),
               format="sparse")
    assert e.value.status == stc.STC_ESINGULAR
