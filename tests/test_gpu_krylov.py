"""GPU parity of the staircase-preconditioned GMRES (stc_solve_gmres) against
the oracle's restarted GMRES (oracle/krylov.py) and the direct solvers.

With krylov_keep_all (every cycle kept, no safeguard) one cycle from the
same start gives the oracle's cycle to 1e-10 in the 1-norm, and three
cycles the oracle's three (the same Krylov steps in exact arithmetic; the
GPU orthogonalises by classical Gram-Schmidt twice, the oracle by modified
Gram-Schmidt).  Converged vectors (||Q^T pi||_1 <= 1e-13) agree with GTH or
level reduction to 1e-10.  The safeguard, the product's own rule for
rejecting stalled cycles, is tested as behaviour: a drifting QBD converges
at the stationary pace, and a chain without drift keeps every cycle.
"""
import numpy as np
import pytest

import synth
from oracle import dense, gth, krylov, level_reduction, staircase

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


CHAINS = [
    ("qbd_L40_m16", lambda: synth.qbd(40, 16, 3, last=9), "dense"),
    ("band_L48_m16", lambda: synth.banded(48, 16, 5, b=2, density=0.3), "dense"),
    ("band_L48_m16_sparse", lambda: synth.banded(48, 16, 5, b=2, density=0.3), "sparse"),
    ("skipfree_L30_m8", lambda: synth.skip_free(30, 8, 4, b=4), "dense"),
    ("loc_L20_m8_any", lambda: synth.localized(20, 8, 9, up=3, down=2, jumps=2, ragged=True),
     "any"),
    # levels of up to 512: the large-block sweep (gather and sliced apply) as the operator
    ("loc_L4_m512_any", lambda: synth.localized(4, 512, 17, up=2, down=1, jumps=1, ragged=True,
                                                density=0.004), "any"),
]


def _solver(g, fmt, **kw):
    from paper_2302_07551_amd import Solver, stc
    if fmt == "any":
        return Solver(None, g.sizes, stc.STC_ANY_PATTERN, csr=g.csr, format="sparse", **kw)
    return Solver(g.blocks, g.sizes, g.b, format=fmt, **kw)


def _system(g, fmt):
    if fmt == "any":
        return staircase.SparseBlockSystem(g.to_scipy(), g.sizes)
    return staircase.BlockSystem(g.blocks, g.sizes, g.b)


def _direct(g, fmt):
    if fmt == "any":
        return gth.gth(g.to_scipy().toarray())
    return level_reduction.level_reduction(g.blocks, g.sizes, g.b)


@pytest.mark.parametrize("stair_type", [1, 2])
@pytest.mark.parametrize("name,make,fmt", CHAINS, ids=[c[0] for c in CHAINS])
def test_gmres_converges_to_the_direct_solution(name, make, fmt, stair_type):
    g = make()
    _say(f"gmres {name} type {stair_type}")
    s = _solver(g, fmt, stair_type=stair_type, krylov_restart=30, poison=True)
    pi, info = s.solve_gmres(tol=1e-13, restart=30, max_applies=20_000)
    assert info["status"] == 0 and info["residual_1"] <= 1e-13
    assert np.abs(pi - _direct(g, fmt)).sum() <= 1e-10
    s.close()


@pytest.mark.parametrize("name,make,fmt", CHAINS, ids=[c[0] for c in CHAINS])
def test_one_cycle_matches_the_oracle(name, make, fmt):
    """Every cycle kept: one cycle's iterate and change against the oracle's
    cycle, element by element."""
    from paper_2302_07551_amd import stc
    g = make()
    r = 12
    s = _solver(g, fmt, krylov_restart=r, krylov_keep_all=True)
    x0 = np.random.default_rng(7).uniform(0.5, 1.5, g.N)
    pi, info = s.solve_gmres(x0, tol=0.0, restart=r, max_applies=r + 1)
    assert info["status"] == stc.STC_EMAXIT and info["iters"] == r + 1
    x0n = x0 / x0.sum()
    cyc, applies, _ = krylov.gmres_cycle(_system(g, fmt), x0n, r)
    err = np.abs(pi - cyc).sum()
    _say(f"one cycle {name}: |pi - oracle cycle|_1 = {err:.2e}")
    assert applies == r + 1 and err <= 1e-10
    assert abs(info["diff_1"] - np.abs(cyc - x0n).sum()) <= 1e-10
    s.close()


@pytest.mark.parametrize("name,make,fmt", [CHAINS[0], CHAINS[2], CHAINS[4]],
                         ids=[CHAINS[k][0] for k in (0, 2, 4)])
def test_three_cycles_match_restarted_gmres(name, make, fmt):
    """Every cycle kept: three restarted cycles against the oracle's plain
    restarted GMRES with the same budget."""
    g = make()
    r = 10
    s = _solver(g, fmt, krylov_restart=r, krylov_keep_all=True)
    x0 = np.random.default_rng(8).uniform(0.5, 1.5, g.N)
    pi, info = s.solve_gmres(x0, tol=0.0, restart=r, max_applies=3 * (r + 1))
    want = krylov.gmres_solve(_system(g, fmt), restart=r, tol=0.0, maxit=3 * (r + 1), x0=x0)
    err = np.abs(pi - want.x).sum()
    _say(f"three cycles {name}: |pi - oracle|_1 = {err:.2e}, residual {info['residual_1']:.2e}")
    assert want.cycles == 3 and info["iters"] == want.applies == 3 * (r + 1)
    assert err <= 1e-10
    assert abs(info["residual_1"] - want.residual) <= 1e-12 + 1e-8 * want.residual
    s.close()


def test_gmres_needs_far_fewer_applies_than_sweeps_and_is_deterministic():
    g = synth.banded(64, 16, 5, b=2, density=0.3)
    s = _solver(g, "dense", krylov_restart=40)
    p1, i1 = s.solve_gmres(tol=1e-12, restart=40)
    p2, i2 = s.solve_gmres(tol=1e-12, restart=40)
    assert i1["iters"] == i2["iters"] and np.array_equal(p1, p2)
    _pi, info = s.solve(tol=1e-12, maxit=200_000)
    s2 = _solver(g, "dense", stop="residual", check_every=50)
    _pi2, info2 = s2.solve(tol=1e-12, maxit=200_000)
    _say(f"applies {i1['iters']} vs stationary sweeps {info2['iters']}")
    assert i1["iters"] * 10 < info2["iters"]
    s.close()
    s2.close()


def test_gmres_argument_errors():
    from paper_2302_07551_amd import stc
    g = synth.qbd(8, 8, 2)
    s = _solver(g, "dense")
    with pytest.raises(stc.StcError) as e:
        s.solve_gmres(restart=4)
    assert e.value.status == stc.STC_EINVAL and "Krylov workspace" in str(e.value)
    s.close()
    s = _solver(g, "dense", krylov_restart=4)
    with pytest.raises(stc.StcError) as e:
        s.solve_gmres(restart=5)
    assert e.value.status == stc.STC_EINVAL
    with pytest.raises(stc.StcError) as e:
        s.solve_gmres(np.full(g.N, -1.0), restart=4)
    assert e.value.status == stc.STC_EINVAL
    s.close()


def test_gmres_mutex_full_size():
    """The mutual-exclusion model at N = 64839 (any block pattern): GMRES to a
    residual of 1e-12 against the closed form."""
    g = synth.mutual_exclusion(16, 12, synth.config_seed(3))
    s = _solver(g, "any", krylov_restart=30)
    pi, info = s.solve_gmres(tol=1e-12, restart=30)
    err = np.abs(pi - synth.mutual_exclusion_pi(g)).sum()
    _say(f"mutex gmres: applies {info['iters']} residual {info['residual_1']:.2e} err {err:.2e}")
    assert info["status"] == 0 and err <= 1e-10
    s.close()


def test_safeguard_on_a_drifting_qbd():
    """Short GMRES cycles stall on a QBD with drift; the safeguard falls back
    to plain steps, so the solve converges in about as many applications as
    the stationary iteration needs sweeps."""
    g = synth.qbd(256, 16, 11)
    s = _solver(g, "dense", krylov_restart=30)
    pi, info = s.solve_gmres(tol=1e-12, restart=30, max_applies=20_000)
    s2 = _solver(g, "dense", stop="residual", check_every=10)
    _p, info2 = s2.solve(tol=1e-12, maxit=100_000)
    _say(f"drifting QBD: applies {info['iters']} vs stationary sweeps {info2['iters']}")
    assert info["status"] == 0
    assert info["iters"] <= 1.5 * info2["iters"]
    assert np.abs(pi - _direct(g, "dense")).sum() <= 1e-10
    s.close()
    s2.close()


def test_gmres_device_vectors_match_host():
    from paper_2302_07551_amd import stc
    g = synth.qbd(24, 16, 31, last=5)
    s = _solver(g, "dense", krylov_restart=20)
    x0 = np.random.default_rng(2).uniform(0.5, 1.5, g.N)
    p_host, i_host = s.solve_gmres(x0, tol=1e-13, restart=20)
    xd = torch.tensor(x0, dtype=torch.float64, device="cuda")
    pd = torch.empty(g.N, dtype=torch.float64, device="cuda")
    info = stc.stc_solve_gmres(s.h, xd, 20, 1e-13, 100_000, pd)
    assert info["iters"] == i_host["iters"]
    assert np.array_equal(pd.cpu().numpy(), p_host)
    s.close()


@pytest.mark.parametrize("name,make,fmt", [CHAINS[1], CHAINS[2], CHAINS[4]],
                         ids=[CHAINS[k][0] for k in (1, 2, 4)])
def test_mixed_gmres_applies_fp32_then_reaches_the_fp64_solution(name, make, fmt):
    """STC_MIXED handles run the first applications of M^{-1} N in FP32 and
    finish in FP64: same direct solution to 1e-10."""
    g = make()
    s = _solver(g, fmt, precision="mixed", krylov_restart=30, switch_tol=1e-7, poison=True)
    pi, info = s.solve_gmres(tol=1e-13, restart=30, max_applies=20_000)
    _say(f"mixed gmres {name}: applies {info['iters']}, fp32 {info['iters_fp32']}")
    assert info["status"] == 0 and 0 < info["iters_fp32"] < info["iters"]
    assert np.abs(pi - _direct(g, fmt)).sum() <= 1e-10
    s.close()


def test_gmres_from_the_solution_and_with_an_unreachable_tol():
    """A start that already meets tol returns at once with no application of
    T; tol = 0 cannot be met, and the solve ends with STC_EMAXIT (a stalled
    Krylov space or a spent budget) with pi and the residual still filled."""
    from paper_2302_07551_amd import stc
    g = synth.qbd(40, 16, 3, last=9)
    s = _solver(g, "dense", krylov_restart=20)
    pi, info = s.solve_gmres(tol=1e-13, restart=20)
    assert info["status"] == 0
    p2, i2 = s.solve_gmres(pi, tol=1e-12, restart=20)
    assert i2["status"] == 0 and i2["iters"] == 0 and i2["residual_1"] <= 1e-12
    assert np.abs(p2 - pi).sum() <= 1e-14
    p3, i3 = s.solve_gmres(pi, tol=0.0, restart=20, max_applies=400)
    _say(f"tol 0: status {i3['status']} applies {i3['iters']} residual {i3['residual_1']:.2e}")
    assert i3["status"] == stc.STC_EMAXIT and 0 < i3["iters"] <= 400
    assert np.isfinite(i3["residual_1"]) and i3["residual_1"] <= 1e-12
    assert np.abs(p3 - _direct(g, "dense")).sum() <= 1e-10
    s.close()


def test_one_cycle_with_unrolled_dot_chunks():
    """A padded vector of 2100 x 64 = 134400 entries gives each of the dot
    kernel's 128 chunks 1050 entries: four terms per thread through the
    unrolled loop and a tail of one for the first 26 threads.  One cycle,
    kept whatever it does, against the oracle's cycle."""
    from paper_2302_07551_amd import stc
    g = synth.qbd(2100, 64, 13)
    r = 8
    s = _solver(g, "dense", krylov_restart=r, krylov_keep_all=True)
    x0 = np.random.default_rng(11).uniform(0.5, 1.5, g.N)
    pi, info = s.solve_gmres(x0, tol=0.0, restart=r, max_applies=r + 1)
    assert info["status"] == stc.STC_EMAXIT and info["iters"] == r + 1
    x0n = x0 / x0.sum()
    cyc, applies, _ = krylov.gmres_cycle(_system(g, "dense"), x0n, r)
    err = np.abs(pi - cyc).sum()
    _say(f"2100 x 64 cycle: |pi - oracle cycle|_1 = {err:.2e}")
    assert applies == r + 1 and err <= 1e-10
    assert abs(info["diff_1"] - np.abs(cyc - x0n).sum()) <= 1e-10
    s.close()


def test_safeguard_keeps_every_cycle_without_drift():
    """On a chain without drift every cycle beats the plain rate, so the
    safeguarded solve takes the same path as the one that keeps every cycle:
    the same applications and bitwise the same vector."""
    g = synth.banded(64, 16, 5, b=2, density=0.3)
    out = []
    for keep_all in (False, True):
        s = _solver(g, "dense", krylov_restart=30, krylov_keep_all=keep_all)
        out.append(s.solve_gmres(tol=1e-12, restart=30))
        s.close()
    (p0, i0), (p1, i1) = out
    _say(f"no drift: applies {i0['iters']} (every cycle kept: {i1['iters']})")
    assert i0["status"] == 0 and i0["iters"] == i1["iters"]
    assert np.array_equal(p0, p1)
