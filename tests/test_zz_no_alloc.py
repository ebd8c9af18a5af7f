"""The allocation-free residual (stc_residual_noalloc, its staging in a static
device array) against stc_residual, through the C ABI: bitwise the same value
on two calls in a row, the second with a smaller input (a banded handle after
a QBD handle, then a generator of any block pattern), and STC_EINVAL with a
clear message for a handle whose staging exceeds the array."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2302_07551_amd import stc
    stc.load_library()


def _noalloc(s, x):
    from paper_2302_07551_amd import stc
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    stc.stc_residual_noalloc(s.h, xd, out)
    s.stream.synchronize()
    return float(out.cpu()[0])


def test_noalloc_residual_equals_stc_residual():
    from paper_2302_07551_amd import Solver, stc
    rng = np.random.default_rng(5)
    cases = [
        ("qbd 1000 x 64", synth.qbd(1000, 64, 5, last=37), "dense"),
        ("banded 30 x 16", synth.banded(30, 16, 6, b=2, density=0.3, last=9), "dense"),
        ("any pattern 20 x 8", synth.localized(20, 8, 9, up=3, down=2, jumps=2, ragged=True),
         "any"),
    ]
    for name, g, fmt in cases:      # each input smaller than the one before
        if fmt == "any":
            s = Solver(None, g.sizes, stc.STC_ANY_PATTERN, csr=g.csr, format="sparse")
        else:
            s = Solver(g.blocks, g.sizes, g.b)
        x = rng.uniform(-0.5, 1.5, g.N)
        want = s.residual(x)
        got = _noalloc(s, x)
        print(f"{name}: stc_residual {want!r}, noalloc {got!r}", flush=True)
        assert got == want
        s.close()


def test_noalloc_residual_on_large_blocks():
    """The large-block residual kernels (levels of 1000 and 512 states,
    column slices of 64) through the allocation-free entry point: bitwise
    stc_residual's value, the second handle smaller than the first."""
    from paper_2302_07551_amd import Solver, stc
    rng = np.random.default_rng(6)
    for m, L, seed in ((1000, 4, 18), (512, 3, 19)):
        g = synth.localized(L, m, seed, up=1, down=1, jumps=1, ragged=True, density=0.003)
        s = Solver(None, g.sizes, stc.STC_ANY_PATTERN, csr=g.csr, format="sparse")
        x = rng.uniform(-0.5, 1.5, g.N)
        want = s.residual(x)
        got = _noalloc(s, x)
        print(f"any pattern {L} x {m}: stc_residual {want!r}, noalloc {got!r}", flush=True)
        assert got == want
        s.close()


def test_noalloc_rejects_staging_above_the_limit():
    from paper_2302_07551_amd import Solver, stc
    L = 600_000                      # padded vector 600000 x 8 x 8 B = 38.4 MB > 32 MiB
    g = synth.birth_death(np.full(L, 0.9), np.full(L, 1.0))
    s = Solver(g.blocks, g.sizes, g.b)
    x = np.full(g.N, 1.0 / g.N)
    with pytest.raises(stc.StcError) as e:
        _noalloc(s, x)
    assert e.value.status == stc.STC_EINVAL and "allocation-free limit" in str(e.value)
    assert np.isfinite(s.residual(x))
    s.close()
