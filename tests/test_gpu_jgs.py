"""Algorithm 1 (JGS: block Jacobi across chunks of levels, block Gauss-Seidel
inside each) on the GPU, the method the paper compares the stair splitting
with, against the oracle's jgs_sweep (pinned by the dense splitting formula).

One sweep from the same x agrees to 1e-13 in the 1-norm (FP64) or 1e-5
(FP32) for one chunk (plain block Gauss-Seidel), a few, and one per level
(block Jacobi); a burst's changes agree with the oracle's; converged solves
of block Gauss-Seidel and JGS reach GTH within 1e-10 with the oracle's sweep
count (within 1).
"""
import numpy as np
import pytest

import synth
from oracle import dense, gth, staircase

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


def _chunks(L, p):
    """The library's split: chunk c holds levels [c L / p, (c + 1) L / p)."""
    return [(c * L // p, (c + 1) * L // p - c * L // p) for c in range(p)]


def _solver(g, p, **kw):
    from paper_2302_07551_amd import Solver
    return Solver(g.blocks, g.sizes, g.b, method="jgs", jgs_chunks=p, **kw)


SHAPES = [
    ("qbd_L40_m16_ragged", lambda: synth.qbd(40, 16, 3, last=9)),
    ("qbd_L9_m8", lambda: synth.qbd(9, 8, 5, last=3)),
    ("band_L30_m16_b2", lambda: synth.banded(30, 16, 11, b=2, density=0.3)),
    ("qbd_L7_m128", lambda: synth.qbd(7, 128, 10, last=100)),
    ("qbd_L12_m64", lambda: synth.qbd(12, 64, 9, last=40)),
    ("skipfree_L20_m8_b4", lambda: synth.skip_free(20, 8, 4, b=4)),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make", SHAPES, ids=[s[0] for s in SHAPES])
def test_one_sweep_matches_the_oracle(name, make, precision):
    g = make()
    sysb = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    x = synth.positive_start(g, 21)
    tol = 1e-13 if precision == "fp64" else 1e-5
    for p in sorted({1, 2, 3, g.L}):
        if p > g.L:
            continue
        s = _solver(g, p, precision=precision)
        z, d = s.step(x)
        zr, dr = staircase.jgs_sweep(sysb, x / x.sum(), _chunks(g.L, p))
        err = np.abs(z - zr).sum()
        _say(f"jgs {name} {precision} p={p}: |z - z_oracle|_1 = {err:.2e}")
        assert err <= tol and abs(d - dr) <= tol, p
        s.close()


@pytest.mark.parametrize("p", [1, 4])
def test_burst_and_its_changes(p):
    g = synth.qbd(64, 16, synth.config_seed(0))
    sysb = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    x = synth.positive_start(g, 3)
    s = _solver(g, p)
    s.load(x)
    diffs = s.sweeps(9, with_diffs=True)
    z = s.store()
    xr = x / x.sum()
    want = []
    for _ in range(9):
        xr, d = staircase.jgs_sweep(sysb, xr, _chunks(g.L, p))
        want.append(d)
    assert np.abs(z - xr).sum() <= 1e-13
    assert np.allclose(diffs, want[:8], rtol=0, atol=1e-13)
    s.close()


def _oracle_solve(g, p, tol, maxit=100000):
    sysb = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    x, it = np.full(g.N, 1.0 / g.N), 0
    while it < maxit:
        x, d = staircase.jgs_sweep(sysb, x, _chunks(g.L, p))
        it += 1
        if d <= tol:
            break
    return x, it


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("p", [1, 2, 8])
def test_converged_solve_reaches_gth(p, precision):
    g = synth.qbd(40, 16, 3, last=9)
    ref = gth.gth(dense.assemble_Q(g.blocks, g.sizes, g.b))
    s = _solver(g, p, precision=precision, check_every=7, switch_tol=1e-6)
    pi, info = s.solve(tol=1e-13, maxit=100000, allow_maxit=False)
    err = np.abs(pi - ref).sum()
    _say(f"jgs p={p} {precision}: sweeps {info['iters']} (fp32 {info['iters_fp32']}), err {err:.2e}")
    assert err <= 1e-10
    if precision == "fp64":
        _x, it = _oracle_solve(g, p, 1e-13)
        assert abs(info["iters"] - it) <= 1
    else:
        assert 0 < info["iters_fp32"] < info["iters"]
    s.close()


def test_block_gauss_seidel_paces_the_stair_splitting():
    """On a block-tridiagonal chain block Gauss-Seidel and the stair splitting
    share their spectrum (section 2), so their sweep counts to the same
    tolerance are close; JGS with more chunks needs more."""
    from paper_2302_07551_amd import Solver
    g = synth.qbd(128, 16, 17)
    counts = {}
    for p in (1, 16):
        s = _solver(g, p, check_every=25)
        _pi, info = s.solve(tol=1e-12, maxit=200000, allow_maxit=False)
        counts[p] = info["iters"]
        s.close()
    s = Solver(g.blocks, g.sizes, g.b, check_every=25)
    _pi, info = s.solve(tol=1e-12, maxit=200000, allow_maxit=False)
    s.close()
    _say(f"sweeps: stair {info['iters']}, BGS {counts[1]}, JGS(16) {counts[16]}")
    assert 0.8 * info["iters"] <= counts[1] <= 1.25 * info["iters"]
    assert counts[16] > counts[1]


def test_jgs_argument_errors():
    from paper_2302_07551_amd import Batch, Solver, stc
    g = synth.qbd(8, 8, 2)
    for kw in ({"jgs_chunks": 0}, {"jgs_chunks": 9}, {"jgs_chunks": 2, "format": "sparse"},
               {"jgs_chunks": 2, "krylov_restart": 4}):
        with pytest.raises(stc.StcError) as e:
            Solver(g.blocks, g.sizes, g.b, method="jgs", **kw)
        assert e.value.status == stc.STC_EINVAL
    s = _solver(g, 2)
    b = Batch(2, 64)
    with pytest.raises(stc.StcError) as e:
        b.set([s], tol=0.0)
    assert e.value.status == stc.STC_EINVAL
    b.close()
    s.close()


def test_profiled_sweeps_then_a_new_setup():
    """Algorithm 1 sweeps in one launch per sweep: the profiled sweeps report
    its time as phase A's and none for phase B, and leave no error behind
    for the next call (a setup right after them succeeds)."""
    from paper_2302_07551_amd import stc
    g = synth.qbd(64, 16, 5)
    s = _solver(g, 4)
    s.load(None)
    ms_a, ms_b, _ms_f, ms = stc.stc_profile_sweeps(s.h, 3)
    assert ms_a > 0.0 and ms_b == 0.0 and ms >= ms_a
    s.close()
    s2 = _solver(g, 8)
    _z, d = s2.step(synth.positive_start(g, 1))
    assert np.isfinite(d)
    s2.close()
