"""Setup in two halves (stc_prepare on the host, stc_setup_prepared on the
device) gives the handle stc_setup gives: the same inverse and blocks, so
the same sweeps bit for bit, in every precision stage."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [
    ("qbd_L33_m8_ragged_fp64", lambda: synth.qbd(33, 8, 31, last=5), "fp64"),
    ("qbd_L40_m24_mixed", lambda: synth.qbd(40, 24, 32), "mixed"),
    ("banded_b2_L24_m64_fp32", lambda: synth.banded(24, 64, 33, b=2, density=0.3), "fp32"),
    ("qbd_L20_m128_ragged_mixed", lambda: synth.qbd(20, 128, 34, last=77), "mixed"),
]


@pytest.mark.parametrize("name,make,precision", CASES, ids=[c[0] for c in CASES])
def test_prepared_setup_sweeps_like_setup(name, make, precision):
    from paper_2302_07551_amd import Prepared, Solver
    g = make()
    print(name, flush=True)
    a = Solver(g.blocks, g.sizes, g.b, precision=precision, switch_tol=1e-6)
    p = Prepared(g.blocks, g.sizes, g.b, precision=precision, switch_tol=1e-6)
    b = Solver.from_prepared(p)
    p.close()                       # the solver no longer needs the host half
    assert b.footprint == a.footprint and b.N == a.N
    for s in (a, b):
        s.load(None)
        s.sweeps(13)
    assert np.array_equal(a.store(), b.store())
    pa, ia = a.solve(tol=1e-12, maxit=20000)
    pb, ib = b.solve(tol=1e-12, maxit=20000)
    assert ia["iters"] == ib["iters"] and np.array_equal(pa, pb)
    a.close()
    b.close()


def test_prepared_setup_finds_a_singular_block():
    from paper_2302_07551_amd import Prepared, Solver, stc
    m = 64
    g = synth.qbd(6, m, 103)
    g.blocks[3, 0] = 0.0
    g.blocks[3, 2] = 0.0
    ar = np.arange(m)
    g.blocks[3, 1, ar, ar] = 0.0
    g.blocks[3, 1, ar, ar] = -g.blocks[3, 1].sum(axis=1)
    p = Prepared(g.blocks, g.sizes, g.b)
    with pytest.raises(stc.StcError) as e:
        Solver.from_prepared(p)
    assert e.value.status == stc.STC_ESINGULAR
    p.close()
    with pytest.raises(ValueError):
        Solver.from_prepared(p)     # released


def test_one_prepared_setup_serves_two_precisions():
    """The host half does not depend on the precision: a setup prepared for
    FP64 sets up a mixed-precision solver equal to one set up directly."""
    from paper_2302_07551_amd import Prepared, Solver, stc
    g = synth.qbd(30, 16, 35)
    p = Prepared(g.blocks, g.sizes, g.b, precision="fp64")
    opt = stc.make_options("mixed", switch_tol=1e-6)
    a = Solver(g.blocks, g.sizes, g.b, precision="mixed", switch_tol=1e-6)
    arena = torch.empty(a.footprint, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    opt.arena, opt.arena_bytes = arena.data_ptr(), a.footprint
    opt.stream = torch.cuda.current_stream().cuda_stream or None
    h = stc.stc_setup_prepared(p.p, opt)
    p.close()
    x = np.empty(a.N)
    for hh in (a.h, h):
        stc.stc_load(hh, None)
        stc.stc_sweeps(hh, 9)
    y = np.empty(a.N)
    stc.stc_store(a.h, x)
    stc.stc_store(h, y)
    assert np.array_equal(x, y)
    stc.stc_destroy(h)
    a.close()
