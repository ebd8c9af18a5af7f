"""GPU parity at the full sizes of the large workloads, in the launch
configuration the benchmark times (launch variant picked by stc_autotune).

- 16384 levels x m = 128 QBD (N = 2,097,152), FP64 and FP32 handles.  A
  whole oracle sweep at this size takes tens of seconds, so outputs are
  sampled: windows of levels spread along the chain, the two ends included,
  give exact unnormalised sweep values (window_oracle.py). They are compared
  with the GPU sweep up to the one normalisation scalar, which e^T z = 1
  pins.  The change the GPU returns is checked against ||z - x||_1 on the
  host, and the FP64 residual at full size against the oracle's.  The same
  sweep as a burst on the resident iterate (the persistent kernel when the
  tuned variant has one) meets the same samples, and a burst of three
  sweeps equals three chained steps.
- Banded 2048 x 128, block bandwidth 2, 10 % density (N = 262144), dense and
  sparse storage, FP64 and FP32: element by element against one whole
  oracle sweep.
"""
import numpy as np
import pytest

import synth
from oracle import dense, staircase
from window_oracle import sampled_stair_apply

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


@pytest.fixture(scope="module")
def large_qbd():
    g = synth.qbd(16384, 128, synth.config_seed(3))
    yield g
    del g


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_large_qbd_sampled_step(large_qbd, precision):
    from paper_2302_07551_amd import Solver, stc
    g = large_qbd
    x = synth.positive_start(g, 17)
    _say(f"16384 x 128 {precision}: setup")
    s = Solver(g.blocks, g.sizes, g.b, precision=precision)
    stc.stc_autotune(s.h, 5)
    stage = stc.STC_FP32 if precision == "fp32" else stc.STC_FP64
    _say(f"16384 x 128 {precision}: variant {stc.stc_get_variant(s.h, stage)}, step")
    z, d = s.step(x)
    idx, u = sampled_stair_apply(g, x)
    zs = z[idx]
    c = u.sum() / zs.sum()          # e^T (M^{-1} N x), the scalar the sweep divided by
    rel = np.abs(c * zs - u).sum() / np.abs(u).sum()
    tol = 1e-13 if precision == "fp64" else 1e-5
    _say(f"16384 x 128 {precision}: {idx.size} sampled states, relative 1-norm {rel:.2e}, "
         f"|e^T z - 1| {abs(z.sum() - 1.0):.2e}")
    assert np.isfinite(c) and c > 0.0
    assert rel <= tol
    assert abs(z.sum() - 1.0) <= (1e-12 if precision == "fp64" else 1e-6)
    assert abs(d - np.abs(z - x).sum()) <= (1e-12 if precision == "fp64" else 1e-5)
    # the same sweep as a burst on the resident iterate (the persistent kernel
    # when the tuned variant has one, as in the benchmark's solves)
    s.load(x)
    s.sweeps(1)
    zb = s.store()
    zbs = zb[idx]
    relb = np.abs((u.sum() / zbs.sum()) * zbs - u).sum() / np.abs(u).sum()
    assert relb <= tol and abs(zb.sum() - 1.0) <= (1e-12 if precision == "fp64" else 1e-6)
    assert np.abs(zb - z).sum() <= tol
    # three sweeps in one burst continue the recurrence of three steps
    s.load(x)
    s.sweeps(3)
    z3 = s.store()
    zz = z
    for _ in range(2):
        zz, _d = s.step(zz)
    _say(f"16384 x 128 {precision}: burst vs step {np.abs(zb - z).sum():.2e}, "
         f"3-sweep burst vs 3 steps {np.abs(z3 - zz).sum():.2e}")
    assert np.abs(z3 - zz).sum() <= tol
    if precision == "fp64":
        r = s.residual(x)
        rr = dense.residual_1(g.blocks, g.sizes, g.b, x)
        _say(f"16384 x 128 residual {r:.6e} vs oracle {rr:.6e}")
        assert abs(r - rr) <= 1e-12 * max(1.0, rr)
    s.close()


@pytest.fixture(scope="module")
def banded_full():
    g = synth.banded(2048, 128, synth.config_seed(2), b=2, density=0.1, decay=0.5)
    x = synth.positive_start(g, 29)
    zr, dr = staircase.staircase_sweep(staircase.BlockSystem(g.blocks, g.sizes, g.b), x, 1)
    return g, x, zr, dr


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("fmt", ["dense", "sparse"])
def test_banded_full_size_step(banded_full, fmt, precision):
    from paper_2302_07551_amd import Solver, stc
    g, x, zr, dr = banded_full
    s = Solver(g.blocks, g.sizes, g.b, format=fmt, precision=precision)
    stc.stc_autotune(s.h, 5)
    z, d = s.step(x)
    err = np.abs(z - zr).sum()
    _say(f"banded 2048 x 128 {fmt} {precision}: |z - zr|_1 = {err:.2e}")
    tol = 1e-13 if precision == "fp64" else 1e-5
    assert err <= tol and abs(d - dr) <= tol
    s.close()
