"""Algorithm 1 (JGS: block Jacobi across chunks of levels, block Gauss-Seidel
inside each) on the GPU, the method the paper compares the stair splitting
with, against the oracle's jgs_sweep (pinned by the dense splitting formula).

One sweep from the same x agrees to 1e-13 in the 1-norm (FP64) or 1e-5
(FP32) for one chunk (plain block Gauss-Seidel), a few, and one per level
(block Jacobi); a burst's changes agree with the oracle's; converged solves
of block Gauss-Seidel and JGS reach GTH within 1e-10 with the oracle's sweep
count (within 1).

Generators of any block pattern (levels up to 256 states, the CSR input)
run the same algorithm from their per-level entry lists, a source read
fresh when its level is one of the chunk's earlier levels: one sweep, bursts
(bit for bit against single sweeps) and converged solves against the same
oracle sweep on the block view of the sparse matrix, and the
mutual-exclusion model against its closed form.
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


# ---------------------------------------------------------------------------
# Algorithm 1 on generators of any block pattern (CSR input, per-level ELL)
# ---------------------------------------------------------------------------
GENERAL = [
    ("loc_L12_m6_ragged", lambda: synth.localized(12, 6, 1, up=2, down=2, jumps=2, ragged=True)),
    ("hess_L16_m8", lambda: synth.localized(16, 8, 2, up=16, down=1, jumps=0)),
    ("loc_L9_m1", lambda: synth.localized(9, 1, 5, up=3, down=3, jumps=1)),
    ("mutex_n10_r6_m32", lambda: synth.mutual_exclusion(10, 6, 4, m=32)),
    ("loc_L7_m128", lambda: synth.localized(7, 128, 7, up=2, down=6, jumps=1, density=0.03)),
    ("loc_L5_m256_ragged", lambda: synth.localized(5, 256, 15, up=2, down=2, jumps=1,
                                                   ragged=True, density=0.02)),
]


def _gen_solver(g, p, **kw):
    from paper_2302_07551_amd import Solver, stc
    return Solver(None, g.sizes, stc.STC_ANY_PATTERN, csr=g.csr, format="sparse", method="jgs",
                  jgs_chunks=p, **kw)


def _gen_system(g):
    return staircase.SparseBlockSystem(g.to_scipy(), g.sizes)


def _gen_start(g, seed):
    x = np.random.default_rng(seed).uniform(0.5, 1.5, g.N)
    return x / x.sum()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make", GENERAL, ids=[s[0] for s in GENERAL])
def test_any_pattern_one_sweep_matches_the_oracle(name, make, precision):
    """One sweep of Algorithm 1 on a pattern of any shape for one chunk
    (block Gauss-Seidel), a few, and one per level (block Jacobi), against
    the oracle's jgs_sweep on the same system."""
    g = make()
    sysg = _gen_system(g)
    x = _gen_start(g, 21)
    tol = 1e-13 if precision == "fp64" else 1e-5
    for p in sorted({1, min(3, g.L), g.L}):
        zr, dr = staircase.jgs_sweep(sysg, x, _chunks(g.L, p))
        s = _gen_solver(g, p, precision=precision, poison=True)
        z, d = s.step(x)
        err = np.abs(z - zr).sum()
        _say(f"jgs any pattern {name} {precision} p={p}: |z - z_oracle|_1 = {err:.2e}")
        assert err <= tol and abs(d - dr) <= tol
        s.close()


@pytest.mark.parametrize("name,make", [GENERAL[k] for k in (0, 3, 5)],
                         ids=[GENERAL[k][0] for k in (0, 3, 5)])
def test_any_pattern_bursts_follow_the_oracle(name, make):
    """Bursts: the iterate and the changes follow the oracle's recurrence,
    and one burst equals bursts of one sweep bit for bit (the flush's
    change kernel has the sweep's geometry)."""
    g = make()
    sysg = _gen_system(g)
    x = _gen_start(g, 5)
    p = min(3, g.L)
    s = _gen_solver(g, p, poison=True)
    s.load(x)
    diffs = s.sweeps(6, with_diffs=True)
    z6 = s.store()
    xr, want = x, []
    for _ in range(6):
        xr, dr = staircase.jgs_sweep(sysg, xr, _chunks(g.L, p))
        want.append(dr)
    assert np.abs(z6 - xr).sum() <= 1e-13
    assert np.abs(np.asarray(diffs) - np.asarray(want[:-1])).max() <= 1e-13
    s.load(x)
    for _ in range(6):
        s.sweeps(1)
    assert np.array_equal(s.store(), z6)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("p", [1, 4])
def test_any_pattern_converged_solve_reaches_gth(p, precision):
    g = synth.localized(12, 8, 9, up=3, down=2, jumps=2, ragged=True)
    ref = gth.gth(g.to_scipy().toarray())
    s = _gen_solver(g, p, precision=precision, check_every=7, switch_tol=1e-6)
    pi, info = s.solve(tol=1e-13, maxit=100000, allow_maxit=False)
    err = np.abs(pi - ref).sum()
    _say(f"jgs any pattern p={p} {precision}: sweeps {info['iters']} "
         f"(fp32 {info['iters_fp32']}), err {err:.2e}")
    assert err <= 1e-10
    if precision == "mixed":
        assert 0 < info["iters_fp32"] < info["iters"]
    s.close()


def test_any_pattern_mutex_closed_form():
    """The mutual-exclusion model (the paper's fourth matrix, N = 4017 here)
    in levels of 256 by block Gauss-Seidel and by JGS over 8 chunks: both
    reach the closed-form stationary vector."""
    g = synth.mutual_exclusion(12, 9, 25, m=256)
    exact = synth.mutual_exclusion_pi(g)
    for p in (1, 8):
        s = _gen_solver(g, p, check_every=50)
        pi, info = s.solve(tol=1e-13, maxit=100000, allow_maxit=False)
        err = np.abs(pi - exact).sum()
        _say(f"jgs mutex m256 p={p}: sweeps {info['iters']}, err {err:.2e}")
        assert err <= 1e-10
        s.close()


LARGE = [
    ("loc_L5_m512_ragged", lambda: synth.localized(5, 512, 17, up=2, down=2, jumps=1, ragged=True,
                                                   density=0.004)),
    ("loc_L4_m1000_ragged", lambda: synth.localized(4, 1000, 18, up=1, down=2, jumps=1,
                                                    ragged=True, density=0.002)),
    ("mutex_n13_r8_m2048", lambda: synth.mutual_exclusion(13, 8, 20, m=2048)),
    ("loc_L18_m512", lambda: synth.localized(18, 512, 27, up=1, down=1, jumps=1, density=0.004)),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make", LARGE, ids=[s[0] for s in LARGE])
def test_large_blocks_one_sweep_matches_the_oracle(name, make, precision):
    """Levels of 512 to 2048 states (a gather and a sliced apply launch per
    level of a chunk): one sweep for p = 1, 2 and L against the oracle.  Steps
    of levels of 1024 or more with under 128 (level, slice) groups split the
    apply over row ranges and add them in a third launch (the 1000 and 2048
    cases, except p = L = 4 at 2048); the 512 cases run unsplit."""
    g = make()
    sysg = _gen_system(g)
    x = _gen_start(g, 22)
    tol = 1e-13 if precision == "fp64" else 1e-5
    for p in sorted({1, 2, g.L}):
        zr, dr = staircase.jgs_sweep(sysg, x, _chunks(g.L, p))
        s = _gen_solver(g, p, precision=precision, poison=True)
        z, d = s.step(x)
        err = np.abs(z - zr).sum()
        _say(f"jgs large blocks {name} {precision} p={p}: |z - z_oracle|_1 = {err:.2e}")
        assert np.all(np.isfinite(z))
        assert err <= tol and abs(d - dr) <= tol
        s.close()


@pytest.mark.parametrize("p", [1, 3])
@pytest.mark.parametrize("k", [0, 1])
def test_large_blocks_bursts_follow_the_oracle(k, p):
    """Bursts on the large blocks (512: one apply launch per step; 1000: the
    row-split apply and its combine): the iterate and the changes follow the
    oracle, and one burst equals bursts of one sweep bit for bit (the flush's
    change kernel takes the apply's (level, slice) slots)."""
    g = LARGE[k][1]()
    sysg = _gen_system(g)
    x = _gen_start(g, 6)
    s = _gen_solver(g, p, poison=True)
    s.load(x)
    diffs = s.sweeps(6, with_diffs=True)
    z6 = s.store()
    xr, want = x, []
    for _ in range(6):
        xr, dr = staircase.jgs_sweep(sysg, xr, _chunks(g.L, p))
        want.append(dr)
    assert np.abs(z6 - xr).sum() <= 1e-13
    assert np.abs(np.asarray(diffs) - np.asarray(want[:-1])).max() <= 1e-13
    s.load(x)
    for _ in range(6):
        s.sweeps(1)
    assert np.array_equal(s.store(), z6)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("p", [1, 2])
def test_large_blocks_mutex_solve_reaches_closed_form(p, precision):
    g = LARGE[2][1]()
    exact = synth.mutual_exclusion_pi(g)
    s = _gen_solver(g, p, precision=precision, check_every=20)
    pi, info = s.solve(tol=1e-13, maxit=100000, allow_maxit=False)
    err = np.abs(pi - exact).sum()
    _say(f"jgs large mutex p={p} {precision}: sweeps {info['iters']} "
         f"(fp32 {info['iters_fp32']}), err {err:.2e}")
    assert err <= 1e-10
    if precision == "mixed":
        assert info["iters_fp32"] > 0
    s.close()


def test_large_blocks_block_jacobi_oscillates_as_the_oracle():
    """With one chunk per level (p = L = 4, block Jacobi) the iteration on
    this block-tridiagonal chain has an eigenvalue -1 and never converges
    (the change stays near 7e-2 in the oracle too), the failure the paper
    reports for JGS as it approaches block Jacobi.  The GPU follows the
    oracle's iterates and changes through 100 sweeps."""
    g = LARGE[2][1]()
    sysg = _gen_system(g)
    x = _gen_start(g, 9)
    s = _gen_solver(g, g.L)
    s.load(x)
    diffs = s.sweeps(100, with_diffs=True)
    z = s.store()
    xr, want = x, []
    for _ in range(100):
        xr, dr = staircase.jgs_sweep(sysg, xr, _chunks(g.L, g.L))
        want.append(dr)
    _say(f"block Jacobi mutex m2048: change {diffs[-1]:.3e} (oracle {want[-2]:.3e}), "
         f"|z - z_oracle|_1 = {np.abs(z - xr).sum():.2e}")
    assert want[-2] > 1e-2
    assert np.abs(z - xr).sum() <= 1e-11
    assert np.abs(np.asarray(diffs) - np.asarray(want[:-1])).max() <= 1e-11
    s.close()


def test_any_pattern_jgs_argument_errors():
    from paper_2302_07551_amd import stc
    g = synth.localized(3, 512, 26, up=1, down=1, jumps=0, density=0.01)
    for kw in ({"jgs_chunks": 0}, {"jgs_chunks": 4}, {"jgs_chunks": 2, "krylov_restart": 4}):
        with pytest.raises(stc.StcError) as e:
            _gen_solver(g, kw.pop("jgs_chunks"), **kw)
        assert e.value.status == stc.STC_EINVAL


def test_full_size_jgs_sweep_matches_the_oracle():
    """The symmetric chain of bandwidth 1135 at its full size (N = 91881, 45
    levels of 2048, as the section 3 comparison builds it): one FP64 sweep of
    block Gauss-Seidel (p = 1, the row-split apply) and of JGS over 12
    chunks (unsplit), element by element against the oracle's sweep of the
    whole chain (its block view is tridiagonal, about 4 GB of dense blocks)."""
    g = synth.banded_random(91881, 1135, 1135, synth.config_seed(3), symmetric=True, m=2048)
    sysg = _gen_system(g)
    x = _gen_start(g, 12)
    for p in (1, 12):
        zr, dr = staircase.jgs_sweep(sysg, x, _chunks(g.L, p))
        s = _gen_solver(g, p)
        z, d = s.step(x)
        err = np.abs(z - zr).sum()
        _say(f"full-size jgs p={p}: |z - z_oracle|_1 = {err:.2e}, change {d:.6e} "
             f"(oracle {dr:.6e})")
        assert err <= 1e-13 and abs(d - dr) <= 1e-13
        s.close()


@pytest.mark.parametrize("p", [1, 3])
def test_large_blocks_profiled_sweeps(p):
    """Profiled Algorithm 1 sweeps on the large blocks (a timed span from the
    first step's gather to the last step's apply or combine): the time is
    reported as phase A's, none for phase B, and the iterate after them is
    the one plain sweeps give."""
    from paper_2302_07551_amd import stc
    g = LARGE[1][1]()
    x = _gen_start(g, 14)
    a, b = _gen_solver(g, p), _gen_solver(g, p)
    a.load(x)
    ms_a, ms_b, _ms_f, ms = stc.stc_profile_sweeps(a.h, 4)
    assert ms_a > 0.0 and ms_b == 0.0 and ms >= ms_a
    b.load(x)
    b.sweeps(4)
    assert np.array_equal(a.store(), b.store())
    a.close()
    b.close()
