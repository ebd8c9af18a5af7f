"""The persistent burst (launch variant bit 2: one cooperative launch per
burst, blocks synchronised by their neighbours' progress flags) runs the same
per-level arithmetic and the same fixed-order reductions as the two launches
per sweep, so every iterate, change and stop sweep must be bitwise equal to
those of the same variant without bit 2."""
import numpy as np
import pytest

import synth
from oracle import level_reduction

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FLOW = 4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(msg):
    print(msg, flush=True)


SHAPES = [
    ("qbd_L64_m16", lambda: synth.qbd(64, 16, synth.config_seed(0))),
    ("qbd_L9_m8_ragged", lambda: synth.qbd(9, 8, 5, last=3)),
    ("qbd_L2_m4", lambda: synth.qbd(2, 4, 6)),
    ("qbd_L3_m4", lambda: synth.qbd(3, 4, 16)),
    ("qbd_L33_m12_pad", lambda: synth.qbd(33, 12, 7, last=7)),
    ("qbd_L301_m32", lambda: synth.qbd(301, 32, 8, last=17)),
    ("qbd_L13_m64", lambda: synth.qbd(13, 64, 9, last=40)),
    ("qbd_L40_m128", lambda: synth.qbd(40, 128, 10, last=100)),
    ("band_L17_m16", lambda: synth.banded(17, 16, 11, b=2, density=0.3)),
    ("band_L203_m32", lambda: synth.banded(203, 32, 13, b=2, density=0.2, last=30)),
    ("bd_L50_m1", lambda: synth.birth_death(np.linspace(0.5, 1.0, 50), np.linspace(1.0, 0.8, 50))),
]


def _sweep_trace(g, precision, stair_type, variant, nsw, x):
    from paper_2302_07551_amd import Solver, stc
    s = Solver(g.blocks, g.sizes, g.b, precision=precision, stair_type=stair_type)
    stage = stc.STC_FP64 if precision == "fp64" else stc.STC_FP32
    stc.stc_set_variant(s.h, stage, variant)
    s.load(x)
    d1 = s.sweeps(nsw, with_diffs=True)
    d2 = s.sweeps(nsw // 3 + 1, with_diffs=True)   # a second burst continues the first
    out = (s.store(), d1, d2, s.query())
    s.close()
    return out


@pytest.mark.parametrize("name,make", SHAPES, ids=[s[0] for s in SHAPES])
@pytest.mark.parametrize("stair_type", [1, 2])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_flow_burst_bitwise_equal(name, make, stair_type, precision):
    g = make()
    x = synth.positive_start(g, 41)
    for v in (0, 3):
        _say(f"flow {name} type {stair_type} {precision} variant {v}|4")
        ref = _sweep_trace(g, precision, stair_type, v, 37, x)
        got = _sweep_trace(g, precision, stair_type, v | FLOW, 37, x)
        assert np.array_equal(got[0], ref[0])
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
        assert got[3][:2] == ref[3][:2]


@pytest.mark.parametrize("name,make", [SHAPES[0], SHAPES[4], SHAPES[5], SHAPES[9]],
                         ids=[SHAPES[k][0] for k in (0, 4, 5, 9)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_flow_solve_stops_at_the_same_sweep(name, make, precision):
    """Converged solves with long bursts (the stop fires inside a burst):
    same stop sweep, same vector, and within 1e-10 of the direct solution."""
    from paper_2302_07551_amd import Solver, stc
    g = make()
    ref = level_reduction.level_reduction(g.blocks, g.sizes, g.b)
    res = []
    for v in (1, 1 | FLOW):
        s = Solver(g.blocks, g.sizes, g.b, precision=precision, check_every=97, switch_tol=1e-6)
        for stage in (stc.STC_FP64, stc.STC_FP32):
            stc.stc_set_variant(s.h, stage, v)
        pi, info = s.solve(tol=1e-13, maxit=200000, allow_maxit=False)
        s.close()
        res.append((pi, info))
        _say(f"solve {name} {precision} variant {v}: {info['iters']} sweeps")
    (p0, i0), (p1, i1) = res
    assert (i1["iters"], i1["iters_fp32"]) == (i0["iters"], i0["iters_fp32"])
    assert np.array_equal(p1, p0)
    # a change below tol bounds the error by about tol / (1 - gamma): 1e-10
    # on the QBDs; the symmetric banded chain mixes slowly (gamma near 1)
    assert np.abs(p1 - ref).sum() <= (1e-10 if g.b == 1 else 2e-9)


def test_flow_residual_stop_and_poisoned_arena():
    from paper_2302_07551_amd import Solver, stc
    g = synth.qbd(77, 16, 55, last=9)
    out = []
    for v in (0, FLOW):
        s = Solver(g.blocks, g.sizes, g.b, stop="residual", check_every=25, poison=True)
        stc.stc_set_variant(s.h, stc.STC_FP64, v)
        out.append(s.solve(tol=1e-12, maxit=100000, allow_maxit=False))
        s.close()
    assert out[0][1]["iters"] == out[1][1]["iters"]
    assert np.array_equal(out[0][0], out[1][0])


def test_flow_full_size_bitwise():
    """The 4096 x 64 FP64 chain in the bench's launch configuration."""
    g = synth.qbd(4096, 64, synth.config_seed(1))
    x = synth.positive_start(g, 3)
    ref = _sweep_trace(g, "fp64", 1, 3, 60, x)
    got = _sweep_trace(g, "fp64", 1, 3 | FLOW, 60, x)
    assert np.array_equal(got[0], ref[0])
    assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])


def test_flow_profile_and_autotune():
    from paper_2302_07551_amd import Solver, stc
    g = synth.qbd(500, 32, 61)
    s = Solver(g.blocks, g.sizes, g.b)
    stc.stc_set_variant(s.h, stc.STC_FP64, FLOW)
    s.load(None)
    ms_a, ms_b, ms_f, ms_s = stc.stc_profile_sweeps(s.h, 20)
    assert ms_a > 0 and ms_a == ms_b and ms_s >= ms_a + ms_b
    assert s.query()[0] == 20
    ms64, _ = stc.stc_autotune(s.h, 5)
    assert ms64 > 0 and 0 <= stc.stc_get_variant(s.h, stc.STC_FP64) < stc.stc_variant_count()
    s.close()
