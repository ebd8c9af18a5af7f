"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Tolerances (FP64): one sweep from the same x agrees to 1e-13 in the 1-norm
(different but exact-in-real-arithmetic ways of applying A_ii^{-1}: explicit
inverse vs LU solve, and different summation orders); converged vectors agree
with the direct reference (GTH / level reduction) to 1e-10; iteration counts
with the oracle's to max(2, 1 %).  FP32 sweeps agree with the FP64 oracle to
1e-5 per sweep (storage rounding of blocks and vector, ~1e-7 relative).
"""
import os

import numpy as np
import pytest

import synth
from oracle import dense, gth, level_reduction, staircase

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_07551_amd import stc
    stc.load_library()


def _solver(g, **kw):
    from paper_2302_07551_amd import Solver
    return Solver(g.blocks, g.sizes, g.b, **kw)


def _say(msg):
    print(msg, flush=True)


SHAPES = [
    # (name, generator factory)
    ("qbd_L64_m16", lambda: synth.qbd(64, 16, synth.config_seed(0))),
    ("qbd_L9_m8_ragged", lambda: synth.qbd(9, 8, 5, last=3)),
    ("qbd_L2_m4", lambda: synth.qbd(2, 4, 6)),
    ("qbd_L33_m12_pad", lambda: synth.qbd(33, 12, 7, last=7)),
    ("qbd_L20_m32", lambda: synth.qbd(20, 32, 8)),
    ("qbd_L13_m64", lambda: synth.qbd(13, 64, 9, last=40)),
    ("qbd_L7_m128", lambda: synth.qbd(7, 128, 10, last=100)),
    ("band_L17_m16", lambda: synth.banded(17, 16, 11, b=2, density=0.3)),
    ("band_L10_m128", lambda: synth.banded(10, 128, 12, b=2, last=77)),
    ("bd_L50_m1", lambda: synth.birth_death(np.linspace(0.5, 1.0, 50), np.linspace(1.0, 0.8, 50))),
]


@pytest.mark.parametrize("name,make", SHAPES, ids=[s[0] for s in SHAPES])
@pytest.mark.parametrize("stair_type", [1, 2])
def test_step_fp64_matches_oracle_sweep(name, make, stair_type):
    g = make()
    _say(f"step fp64 {name} type {stair_type}")
    x = synth.positive_start(g, 123)
    s = _solver(g, stair_type=stair_type)
    z, d = s.step(x)
    zr, dr = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x,
                                       stair_type)
    assert np.abs(z - zr).sum() <= 1e-13
    assert abs(d - dr) <= 1e-13
    s.close()


@pytest.mark.parametrize("name,make", SHAPES[:8], ids=[s[0] for s in SHAPES[:8]])
def test_step_fp32_matches_oracle_sweep(name, make):
    g = make()
    _say(f"step fp32 {name}")
    x = synth.positive_start(g, 321)
    s = _solver(g, precision="fp32")
    z, d = s.step(x)
    zr, dr = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x, 1)
    assert np.abs(z - zr).sum() <= 1e-5
    assert abs(d - dr) <= 1e-5
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make", [SHAPES[0], SHAPES[5], SHAPES[6], SHAPES[8]],
                         ids=[SHAPES[k][0] for k in (0, 5, 6, 8)])
def test_every_launch_variant_matches_oracle(name, make, precision):
    from paper_2302_07551_amd import stc
    g = make()
    x = synth.positive_start(g, 77)
    zr, dr = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x, 1)
    s = _solver(g, precision=precision)
    stage = stc.STC_FP64 if precision == "fp64" else stc.STC_FP32
    tol = 1e-13 if precision == "fp64" else 1e-5
    for v in range(stc.stc_variant_count()):
        _say(f"variant {v} {name} {precision}")
        stc.stc_set_variant(s.h, stage, v)
        z, d = s.step(x)
        assert np.abs(z - zr).sum() <= tol, v
        assert abs(d - dr) <= tol, v
    s.close()


def test_autotune_keeps_results():
    from paper_2302_07551_amd import stc
    g = synth.qbd(64, 16, synth.config_seed(0))
    s = _solver(g, precision="mixed", stop="residual", check_every=4)
    ms64, ms32 = stc.stc_autotune(s.h, 5)
    assert ms64 > 0 and ms32 > 0
    for stage in (stc.STC_FP64, stc.STC_FP32):
        assert 0 <= stc.stc_get_variant(s.h, stage) < stc.stc_variant_count()
    ref = gth.gth(dense.assemble_Q(g.blocks, g.sizes, g.b))
    pi, info = s.solve(tol=1e-12, maxit=100000, allow_maxit=False)
    assert np.abs(pi - ref).sum() <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("name,make", [SHAPES[0], SHAPES[1], SHAPES[2], SHAPES[5],
                                       SHAPES[7], SHAPES[8]],
                         ids=[SHAPES[k][0] for k in (0, 1, 2, 5, 7, 8)])
def test_poisoned_arena(name, make, precision):
    """Every byte of the arena starts as NaN; nothing the library reads before
    writing may leak into a result (both even and odd level counts, so the
    last level is a phase-A level in one case and a phase-B level in the
    other)."""
    from paper_2302_07551_amd import stc
    for g in (make(), synth.qbd(60, 64, 323523084)):
        x = synth.positive_start(g, 13)
        zr, dr = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x, 1)
        stage = stc.STC_FP64 if precision == "fp64" else stc.STC_FP32
        for v in range(stc.stc_variant_count()):
            s = _solver(g, precision=precision, poison=True)
            stc.stc_set_variant(s.h, stage, v)
            z, d = s.step(x)
            tol = 1e-13 if precision == "fp64" else 1e-5
            assert np.all(np.isfinite(z)), (name, v)
            assert np.abs(z - zr).sum() <= tol and abs(d - dr) <= tol, (name, v)
            assert np.isfinite(s.residual(x))
            s.close()


SPARSE = [
    ("band_L16_m128", lambda: synth.banded(16, 128, 21, b=2)),
    ("band_L9_m32_ragged", lambda: synth.banded(9, 32, 22, b=2, density=0.2, last=19)),
    ("band_L12_m8", lambda: synth.banded(12, 8, 23, b=2, density=0.4)),
    ("qbd_L15_m64", lambda: synth.qbd(15, 64, 24, last=50)),
    ("qbd_L8_m16", lambda: synth.qbd(8, 16, 25)),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("stair_type", [1, 2])
@pytest.mark.parametrize("name,make", SPARSE, ids=[s[0] for s in SPARSE])
def test_sparse_format_step_matches_oracle(name, make, stair_type, precision):
    g = make()
    x = synth.positive_start(g, 31)
    zr, dr = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x,
                                       stair_type)
    s = _solver(g, precision=precision, stair_type=stair_type, format="sparse", poison=True)
    z, d = s.step(x)
    tol = 1e-13 if precision == "fp64" else 1e-5
    assert np.all(np.isfinite(z))
    assert np.abs(z - zr).sum() <= tol and abs(d - dr) <= tol
    s.close()


def test_sparse_format_converged_and_fewer_bytes():
    from paper_2302_07551_amd import stc
    g, pstar = synth.planted_reversible(20, 32, 57, b=2, density=0.15)
    dense = _solver(g)
    sparse = _solver(g, format="sparse")
    pi_d, info_d = dense.solve(tol=1e-15, maxit=100000, allow_maxit=False)
    pi_s, info_s = sparse.solve(tol=1e-15, maxit=100000, allow_maxit=False)
    assert np.abs(pi_s - pstar).sum() <= 1e-10
    assert abs(info_s["iters"] - info_d["iters"]) <= 1
    a_d, b_d = stc.stc_phase_bytes(dense.h)
    a_s, b_s = stc.stc_phase_bytes(sparse.h)
    assert a_s + b_s < a_d + b_d
    dense.close()
    sparse.close()


def test_batch_rejects_sparse_chains():
    from paper_2302_07551_amd import Batch, stc
    g = synth.banded(8, 16, 58, b=2)
    s = _solver(g, format="sparse")
    b = Batch(4, 256, b=2)
    with pytest.raises(stc.StcError) as e:
        b.set([s], tol=0.0)
    assert e.value.status == stc.STC_EINVAL
    b.close()
    s.close()


def test_repeated_steps_track_oracle():
    g = synth.qbd(24, 16, 31, last=9)
    s = _solver(g)
    sysb = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    x = synth.positive_start(g, 5)
    xr = x.copy()
    for _ in range(25):
        x, _ = s.step(x)
        xr, _ = staircase.staircase_sweep(sysb, xr, 1)
    assert np.abs(x - xr).sum() <= 1e-12
    s.close()


def test_small_config_converged_parity():
    """64 levels x m=16, stop ||Q^T x||_1 < 1e-12 (the small QBD workload)."""
    g = synth.qbd(64, 16, synth.config_seed(0))
    ref = gth.gth(dense.assemble_Q(g.blocks, g.sizes, g.b))
    s = _solver(g, stop="residual", check_every=1)
    pi, info = s.solve(tol=1e-12, maxit=100000, allow_maxit=False)
    o = staircase.staircase_solve(g.blocks, g.sizes, g.b, tol=1e-12, maxit=100000,
                                  stop=staircase.STOP_RESIDUAL)
    _say(f"C0: gpu iters {info['iters']} oracle {o.iters} err {np.abs(pi - ref).sum():.2e}")
    assert np.abs(pi - ref).sum() <= 1e-10
    assert info["residual_1"] <= 1e-12
    assert abs(info["iters"] - o.iters) <= max(2, 0.01 * o.iters)
    assert abs(dense.residual_1(g.blocks, g.sizes, g.b, pi) - info["residual_1"]) <= 1e-14


@pytest.mark.parametrize("stair_type", [1, 2])
def test_diff_stop_iteration_count_exact(stair_type):
    g = synth.qbd(40, 8, 41, last=5)
    s = _solver(g, stair_type=stair_type, check_every=7)
    pi, info = s.solve(tol=1e-11, maxit=20000, allow_maxit=False)
    o = staircase.staircase_solve(g.blocks, g.sizes, g.b, stair_type=stair_type, tol=1e-11,
                                  maxit=20000)
    assert abs(info["iters"] - o.iters) <= 1
    assert np.abs(pi - o.x).sum() <= 1e-12
    ref = level_reduction.level_reduction(g.blocks, g.sizes, g.b)
    assert np.abs(pi - ref).sum() <= 1e-9


def test_banded_converged_parity():
    """Block-pentadiagonal chain with a planted stationary vector.  Its rates
    are large (q = w / pi), so ||Q^T pi*||_1 itself is ~8e-13 and a residual
    stop below that cannot be met; stop on the change instead."""
    g, pstar = synth.planted_reversible(24, 16, 51, b=2)
    s = _solver(g, stop="diff", check_every=5)
    pi, info = s.solve(tol=1e-15, maxit=200000, allow_maxit=False)
    o = staircase.staircase_solve(g.blocks, g.sizes, g.b, tol=1e-15, maxit=200000)
    assert np.abs(pi - pstar).sum() <= 1e-10
    assert abs(info["iters"] - o.iters) <= max(2, 0.01 * o.iters)


@pytest.mark.parametrize("precision", ["mixed", "fp32"])
def test_reduced_precision_solve(precision):
    g = synth.qbd(48, 16, 61)
    ref = level_reduction.level_reduction(g.blocks, g.sizes, g.b)
    s = _solver(g, precision=precision, stop="residual", check_every=4, switch_tol=1e-6)
    if precision == "mixed":
        pi, info = s.solve(tol=1e-12, maxit=50000, allow_maxit=False)
        _say(f"mixed: iters {info['iters']} fp32 {info['iters_fp32']} err {np.abs(pi - ref).sum():.2e}")
        assert np.abs(pi - ref).sum() <= 1e-10
        assert 0 < info["iters_fp32"] < info["iters"]
    else:
        pi, info = s.solve(tol=1e-6, maxit=2000)
        assert np.abs(pi - ref).sum() <= 1e-4
        assert info["iters_fp32"] == info["iters"]


@pytest.mark.parametrize("tol", [1e-5, 1e-6, 1e-9])
def test_mixed_switch_inside_a_burst_equals_one_sweep_bursts(tol):
    """The FP32 stage's device test fires two sweeps after the change it
    tests, and the sweeps queued behind it in a burst overwrite older FP32
    buffers before the switch.  The FP64 stage must not test changes read
    from them.  A solve with bursts of 50 sweeps gives bitwise the result of
    bursts of one sweep (where nothing runs past the stop), with at least one
    FP64 sweep after the switch, also when tol >= switch_tol."""
    g = synth.qbd(48, 16, 61)
    out = []
    for ce in (1, 50):
        s = _solver(g, precision="mixed", stop="diff", check_every=ce, switch_tol=1e-6)
        out.append(s.solve(tol=tol, maxit=50000, allow_maxit=False))
        s.close()
    (p1, i1), (p50, i50) = out
    _say(f"mixed tol {tol}: iters {i50['iters']} fp32 {i50['iters_fp32']} "
         f"(bursts of one: {i1['iters']} / {i1['iters_fp32']})")
    assert i50["iters"] > i50["iters_fp32"] > 0
    assert (i50["iters"], i50["iters_fp32"]) == (i1["iters"], i1["iters_fp32"])
    assert np.array_equal(p1, p50)
    assert i50["diff_1"] <= tol
    # pi is the oracle's iterate of that sweep, up to the FP32 stage's rounding
    o = staircase.staircase_solve(g.blocks, g.sizes, g.b, tol=0.0, maxit=i50["iters"])
    assert np.abs(p50 - o.x).sum() <= 1e-5


@pytest.mark.parametrize("check_every", [1, 50])
def test_mixed_switch_at_the_fp32_floor(check_every):
    """A switch tolerance below what FP32 sweeps can reach: the FP32 stage
    ends at its rounding floor (its change stops making new lows) instead of
    running to maxit, and the FP64 stage converges to the direct solution."""
    g = synth.qbd(48, 16, 61)
    ref = level_reduction.level_reduction(g.blocks, g.sizes, g.b)
    s = _solver(g, precision="mixed", stop="diff", check_every=check_every, switch_tol=1e-15)
    pi, info = s.solve(tol=1e-13, maxit=50000, allow_maxit=False)
    err = np.abs(pi - ref).sum()
    _say(f"floor switch, bursts of {check_every}: iters {info['iters']} "
         f"fp32 {info['iters_fp32']} err {err:.2e}")
    assert info["status"] == 0 and err <= 1e-10
    assert 0 < info["iters_fp32"] < info["iters"] < 50000
    s.close()


def test_residual_matches_oracle():
    g = synth.banded(12, 32, 71, b=2, last=20)
    x = np.random.default_rng(3).standard_normal(g.N)
    s = _solver(g)
    r = s.residual(x)
    assert abs(r - dense.residual_1(g.blocks, g.sizes, g.b, x)) <= 1e-12 * max(1.0, r)


def test_large_qbd_step_parity_full_size():
    """4096 levels x m=64 (the bandwidth workload) in the launch configuration
    the benchmark times: one full sweep against the oracle sweep."""
    g = synth.qbd(4096, 64, synth.config_seed(1))
    x = synth.positive_start(g, 9)
    s = _solver(g)
    z, d = s.step(x)
    zr, dr = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x, 1)
    _say(f"C1 step: |z-zr|_1 = {np.abs(z - zr).sum():.2e}")
    assert np.abs(z - zr).sum() <= 1e-13
    assert abs(d - dr) <= 1e-13
    # sweeps on the resident iterate continue the same recurrence
    s.load(x)
    s.sweeps(3)
    z3 = s.store()
    xr = x
    for _ in range(3):
        xr, _ = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), xr, 1)
    assert np.abs(z3 - xr).sum() <= 1e-13
    s.close()


def test_deterministic_bitwise():
    g = synth.qbd(64, 16, 81)
    a = _solver(g)
    p1, i1 = a.solve(tol=1e-12, maxit=10000)
    p2, i2 = a.solve(tol=1e-12, maxit=10000)
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(p1, p2)


@pytest.mark.parametrize("format", ["dense", "sparse"])
def test_profiled_sweeps_equal_plain_sweeps(format):
    """The measurement path (dispatch-attached events) runs the same sweeps:
    the iterate and the device's sweep count match plain stc_sweeps bitwise,
    and the phase times are positive and fit inside the sweep time."""
    from paper_2302_07551_amd import stc
    g = synth.qbd(40, 32, 83, last=20)
    a, b = _solver(g, format=format), _solver(g, format=format)
    a.load(None)
    b.load(None)
    a.sweeps(7)
    ms_a, ms_b, ms_f, ms_s = stc.stc_profile_sweeps(b.h, 7)
    assert np.array_equal(a.store(), b.store())
    assert a.query()[0] == b.query()[0] == 7
    assert ms_a > 0 and ms_b > 0 and ms_f >= 0
    assert ms_a + ms_b <= ms_s * 1.001 + 1e-3
    a.close()
    b.close()


def test_device_pointers_match_host():
    g = synth.qbd(16, 16, 91, last=11)
    from paper_2302_07551_amd import stc
    s = _solver(g)
    x = synth.positive_start(g, 2)
    z_host, d_host = s.step(x)
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    zd = torch.empty_like(xd)
    d_dev = stc.stc_step(s.h, xd, zd)
    assert np.array_equal(zd.cpu().numpy(), z_host) and d_dev == d_host
    pid = torch.empty_like(xd)
    info = stc.stc_solve(s.h, xd, 1e-12, 5000, pid)
    pih, info_h = s.solve(x0=x, tol=1e-12, maxit=5000)
    assert np.array_equal(pid.cpu().numpy(), pih) and info["iters"] == info_h["iters"]


# ---------------------------------------------------------------------------
# error paths (inputs that the host or the kernels' own checks turn into codes)
# ---------------------------------------------------------------------------
def test_not_a_generator():
    from paper_2302_07551_amd import stc
    g = synth.qbd(6, 4, 101)
    g.blocks[2, 2, 1, 0] = -0.5
    with pytest.raises(stc.StcError) as e:
        _solver(g)
    assert e.value.status == stc.STC_ENOTGEN
    g = synth.qbd(6, 4, 102)
    g.blocks[3, 1, 0, 0] += 0.25
    with pytest.raises(stc.StcError) as e:
        _solver(g)
    assert e.value.status == stc.STC_ENOTGEN


@pytest.mark.parametrize("m", [4, 64, 128])
def test_singular_diagonal_block(m):
    """A level that never leaves itself: caught by the pivot test of the
    VALU inverse (m <= 16) and of the MFMA blocked inverse (m >= 32)."""
    from paper_2302_07551_amd import stc
    g = synth.qbd(6, m, 103)
    # level 3 never leaves itself: drop its up and down rates, refix the diagonal
    g.blocks[3, 0] = 0.0
    g.blocks[3, 2] = 0.0
    ar = np.arange(m)
    g.blocks[3, 1, ar, ar] = 0.0
    g.blocks[3, 1, ar, ar] = -g.blocks[3, 1].sum(axis=1)
    with pytest.raises(stc.StcError) as e:
        _solver(g)
    assert e.value.status == stc.STC_ESINGULAR


def test_bad_start_vector():
    from paper_2302_07551_amd import stc
    g = synth.qbd(6, 4, 104)
    s = _solver(g)
    x = np.full(g.N, 1.0 / g.N)
    x[3] = -0.1
    with pytest.raises(stc.StcError) as e:
        s.solve(x0=x)
    assert e.value.status == stc.STC_EINVAL
    x[3] = np.nan
    with pytest.raises(stc.StcError) as e:
        s.solve(x0=x)
    assert e.value.status == stc.STC_EINVAL


def test_degenerate_start():
    from paper_2302_07551_amd import stc
    g = synth.qbd(6, 4, 105)
    s = _solver(g)
    x = np.zeros(g.N)
    x[:4] = 0.25          # level 0 only: a phase-A level of stair type 1
    with pytest.raises(stc.StcError) as e:
        s.step(x)
    assert e.value.status == stc.STC_EDEGENERATE


def test_maxit_returns_last_iterate():
    from paper_2302_07551_amd import stc
    g = synth.qbd(30, 8, 106)
    s = _solver(g)
    pi, info = s.solve(tol=1e-30, maxit=37)
    assert info["status"] == stc.STC_EMAXIT and info["iters"] == 37
    o = staircase.staircase_solve(g.blocks, g.sizes, g.b, tol=1e-30, maxit=37)
    assert np.abs(pi - o.x).sum() <= 1e-13
    assert abs(info["diff_1"] - o.err) <= 1e-13


# ---- CSR input: the same packed blocks as dense input, bitwise ------------

CSR_SHAPES = [
    ("qbd_L33_m12_pad", lambda: synth.qbd(33, 12, 7, last=7)),
    ("qbd_L13_m64", lambda: synth.qbd(13, 64, 9, last=40)),
    ("band_L17_m16", lambda: synth.banded(17, 16, 11, b=2, density=0.3)),
    ("band_L10_m128", lambda: synth.banded(10, 128, 12, b=2, last=77)),
]


@pytest.mark.parametrize("name,make", CSR_SHAPES, ids=[c[0] for c in CSR_SHAPES])
@pytest.mark.parametrize("format", ["dense", "sparse"])
def test_csr_input_equals_dense_input(name, make, format):
    """A generator given in CSR form (with stored zeros, and with the
    diagonal left out and recomputed) solves to the bitwise same vector in
    the same number of sweeps as its dense blocks."""
    from paper_2302_07551_amd import Solver
    g = make()
    _say(f"csr {name} {format}")
    ref = _solver(g, format=format)
    pi_ref, info_ref = ref.solve(tol=1e-12, maxit=20000)
    ref.close()
    ip, ix, v = g.to_csr(explicit_zeros=25, seed=3)
    s = Solver(None, g.sizes, g.b, csr=(ip, ix, v), m=g.m, format=format)
    pi, info = s.solve(tol=1e-12, maxit=20000)
    s.close()
    assert info["iters"] == info_ref["iters"]
    assert np.array_equal(pi, pi_ref)
    # diagonal left out of the CSR and recomputed, against dense + recompute
    ref = _solver(g, format=format, recompute_diagonal=True)
    pi_ref, info_ref = ref.solve(tol=1e-12, maxit=20000)
    ref.close()
    ip, ix, v = g.to_csr(drop_diagonal=True)
    s = Solver(None, g.sizes, g.b, csr=(ip, ix, v), m=g.m, format=format,
               recompute_diagonal=True)
    pi, info = s.solve(tol=1e-12, maxit=20000)
    s.close()
    assert info["iters"] == info_ref["iters"]
    assert np.array_equal(pi, pi_ref)


def test_csr_from_scipy_large_threaded():
    """A CSR input large enough for threaded scattering (several packing
    chunks): one sweep matches the oracle, and the solve matches dense input."""
    import scipy.sparse as sps
    from paper_2302_07551_amd import Solver
    g = synth.qbd(1500, 64, 97)                   # 147 MB of blocks, 3 chunks of levels
    ip, ix, v = g.to_csr()
    Q = sps.csr_matrix((v, ix, ip), shape=(g.N, g.N))
    s = Solver.from_sparse(Q, g.sizes, g.b)
    d = _solver(g)
    x = synth.positive_start(g, 5)
    z_csr, z_dense = s.step(x), d.step(x)
    assert np.array_equal(z_csr[0], z_dense[0])
    sysm = staircase.BlockSystem(g.blocks, g.sizes, g.b)
    z_ref, _ = staircase.staircase_sweep(sysm, x, 1)
    assert np.abs(z_csr[0] - z_ref).sum() <= 1e-13
    s.close()
    d.close()


# ---- wide block bands (b = 3, 4): skip-free, banded and planted ----------

WIDE = [
    ("skipfree_b3_L19_m12", lambda: synth.skip_free(19, 12, 71, b=3, last=5)),
    ("skipfree_b4_L23_m32", lambda: synth.skip_free(23, 32, 72, b=4)),
    ("band_b3_L15_m8", lambda: synth.banded(15, 8, 73, b=3, density=0.4, last=3)),
    ("planted_b4_L18_m6", lambda: synth.planted_reversible(18, 6, 74, b=4)[0]),
]


@pytest.mark.parametrize("name,make", WIDE, ids=[w[0] for w in WIDE])
@pytest.mark.parametrize("stair_type", [1, 2])
@pytest.mark.parametrize("format", ["dense", "sparse"])
def test_wide_band_step_matches_oracle(name, make, stair_type, format):
    g = make()
    _say(f"wide step {name} type {stair_type} {format}")
    x = synth.positive_start(g, 19)
    zr, dr = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x,
                                       stair_type)
    for precision, tol in (("fp64", 1e-13), ("fp32", 1e-5)):
        s = _solver(g, stair_type=stair_type, format=format, precision=precision)
        z, d = s.step(x)
        s.close()
        assert np.abs(z - zr).sum() <= tol, precision
        assert abs(d - dr) <= tol, precision


@pytest.mark.parametrize("name,make", WIDE, ids=[w[0] for w in WIDE])
def test_wide_band_converged_and_every_variant(name, make):
    """Solves to the direct solution in both storages; every launch variant
    (the persistent ones fall back to per-phase launches for b > 2) gives
    the same sweep."""
    from paper_2302_07551_amd import stc
    g = make()
    ref = level_reduction.level_reduction(g.blocks, g.sizes, g.b)
    for format in ("dense", "sparse"):
        s = _solver(g, format=format)
        pi, info = s.solve(tol=1e-14, maxit=200000, allow_maxit=False)
        s.close()
        _say(f"wide solve {name} {format}: {info['iters']} sweeps")
        assert np.abs(pi - ref).sum() <= 1e-10
    x = synth.positive_start(g, 23)
    s = _solver(g)
    zs = []
    for v in range(stc.stc_variant_count()):
        stc.stc_set_variant(s.h, stc.STC_FP64, v)
        zs.append(s.step(x)[0])
    s.close()
    for v in range(4, stc.stc_variant_count()):
        assert np.array_equal(zs[v], zs[v - 4]), v


def test_wide_band_batch_equals_alone():
    from paper_2302_07551_amd import Batch, stc
    gens = [synth.skip_free(40 + 9 * k, m, 80 + k, b=4, last=3 if k % 2 else None)
            for k, m in enumerate((8, 16, 32, 64, 12))]
    xs = [synth.positive_start(g, 5 + k) for k, g in enumerate(gens)]
    alone = []
    for g, x in zip(gens, xs):
        s = _solver(g)
        stc.stc_set_variant(s.h, stc.STC_FP64, 0)
        s.load(x)
        s.sweeps(31)
        alone.append(s.store())
        s.close()
    sol = [_solver(g) for g in gens]
    for s, x in zip(sol, xs):
        s.load(x)
    b = Batch(8, 4096, b=4)
    b.set(sol, tol=0.0)
    b.sweeps(31)
    b.sync()
    for k, s in enumerate(sol):
        assert np.array_equal(s.store(), alone[k]), k
        s.close()
    b.close()
