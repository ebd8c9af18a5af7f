"""CPU checks of the boundary: the library loads, exports every symbol the
header declares, and the host-side validation rejects bad input without a GPU
(no kernel is launched on these paths)."""
import os
import re

import numpy as np
import pytest

import synth
from paper_2302_07551_amd import build as hipbuild
from paper_2302_07551_amd import stc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(stc.LIB_PATH):
        hipbuild.build()
    return stc.load_library()


def _declared():
    text = open(os.path.join(ROOT, "include", "stc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(stc.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in range(8):
        assert lib.stc_status_string(code).decode().startswith("STC_")


def _gen_opt(g, **kw):
    gen, keep = stc.make_generator(g.blocks, g.sizes, g.b)
    opt = stc.make_options(**kw)
    return gen, opt, keep


def test_footprint_formula(lib):
    g = synth.qbd(10, 12, 1)
    gen, opt, _ = _gen_opt(g)
    fp64 = stc.stc_footprint_bytes(gen, opt)
    MP, NB, L = 16, 3, 10
    assert fp64 >= L * NB * MP * MP * 8 + L * MP * MP * 8
    gen, opt, _ = _gen_opt(g, precision="mixed")
    mixed = stc.stc_footprint_bytes(gen, opt)
    assert mixed >= fp64 + L * NB * MP * MP * 4


def test_footprint_rejects_bad_shapes(lib):
    g = synth.qbd(4, 4, 2)
    gen, opt, _ = _gen_opt(g)
    gen.L = 1
    assert stc.stc_footprint_bytes(gen, opt) == 0
    gen.L, gen.m = 4, 200
    assert stc.stc_footprint_bytes(gen, opt) == 0
    gen.m, gen.b = 4, 5
    assert stc.stc_footprint_bytes(gen, opt) == 0
    gen.b = 0
    assert stc.stc_footprint_bytes(gen, opt) == 0


def test_setup_rejects_small_arena_before_touching_the_device(lib):
    g = synth.qbd(4, 4, 3)
    gen, opt, _ = _gen_opt(g)
    opt.arena = 4096
    opt.arena_bytes = 16
    with pytest.raises(stc.StcError) as e:
        stc.stc_setup(gen, opt)
    assert e.value.status == stc.STC_ENOMEM


def test_setup_rejects_bad_arguments(lib):
    g = synth.qbd(4, 4, 3)
    gen, opt, _ = _gen_opt(g, stair_type=3)
    opt.arena, opt.arena_bytes = 4096, 1 << 30
    with pytest.raises(stc.StcError) as e:
        stc.stc_setup(gen, opt)
    assert e.value.status == stc.STC_EINVAL
    gen, opt, _ = _gen_opt(g)
    opt.arena, opt.arena_bytes = 4096 + 8, 1 << 30
    with pytest.raises(stc.StcError) as e:
        stc.stc_setup(gen, opt)
    assert e.value.status == stc.STC_EINVAL and "aligned" in str(e.value)


def test_make_generator_checks_shape():
    with pytest.raises(ValueError):
        stc.make_generator(np.zeros((4, 3, 4, 5)), None, 1)


def test_package_public_names_import():
    import paper_2302_07551_amd as p
    for name in ("Batch", "Solver", "StcError", "load_library"):
        assert hasattr(p, name), name
    for name in stc.EXPORTS:
        assert callable(getattr(stc, name, None)) or name in ("stc_status_string",
                                                              "stc_last_error"), name


def test_sparse_footprint_is_smaller(lib):
    g = synth.banded(12, 64, 5, b=2, density=0.1)
    gen, keep = stc.make_generator(g.blocks, g.sizes, g.b)
    dense = stc.stc_footprint_bytes(gen, stc.make_options(format="dense"))
    sparse = stc.stc_footprint_bytes(gen, stc.make_options(format="sparse"))
    assert 0 < dense < sparse    # sparse keeps the dense copies for the residual, plus ELL
    nb, MP = 5, 64
    ell_upper = 12 * 4 * MP * MP * 9
    assert sparse - dense <= ell_upper
    assert stc.stc_footprint_bytes(gen, stc.make_options(format=7)) == 0


def _bad_gen_status(blocks, sizes, b):
    gen, keep = stc.make_generator(blocks, sizes, b)
    opt = stc.make_options()
    opt.arena, opt.arena_bytes = 4096, 1 << 40    # never touched: validation fails first
    with pytest.raises(stc.StcError) as e:
        stc.stc_setup(gen, opt)
    return e.value


def test_threaded_validation_reports_the_first_bad_level(lib):
    """Validation of a large generator is split over host threads; the error
    reported is still the one at the lowest level, as a serial scan finds."""
    g = synth.qbd(600, 64, 31)                     # 59 MB of blocks: several threads
    blocks = g.blocks.copy()
    blocks[500, 0, 3, 5] = -1.0                    # a negative rate, late level
    blocks[101, 2, 7, 1] = np.nan                  # earlier level, another range
    err = _bad_gen_status(blocks, g.sizes, g.b)
    assert err.status == stc.STC_ENOTGEN and "level 101 row 7" in str(err), str(err)
    blocks = g.blocks.copy()
    blocks[450, 1, 9, 9] += 0.5                    # row sum not 0
    blocks[599, 0, 0, 1] = -2.0
    err = _bad_gen_status(blocks, g.sizes, g.b)
    assert err.status == stc.STC_ENOTGEN and "row 9 of level 450" in str(err), str(err)


# ---- CSR input -------------------------------------------------------------

def _csr_gen(g, **kw):
    ip, ix, v = g.to_csr(**{k: kw.pop(k) for k in ("drop_diagonal", "explicit_zeros") if k in kw})
    gen, keep = stc.make_generator_csr(ip, ix, v, g.sizes, g.b, g.m, **kw)
    return gen, keep


CSR_CASES = [
    ("qbd_ragged", lambda: synth.qbd(33, 12, 7, last=7)),
    ("band_b2", lambda: synth.banded(17, 16, 11, b=2, density=0.3, last=9)),
    ("band_m128", lambda: synth.banded(6, 128, 12, b=2, density=0.1)),
]


@pytest.mark.parametrize("name,make", CSR_CASES, ids=[c[0] for c in CSR_CASES])
@pytest.mark.parametrize("fmt", ["dense", "sparse"])
def test_csr_footprint_equals_dense_input(lib, name, make, fmt):
    """The CSR form of a generator needs the same device bytes as its dense
    blocks, also with stored zeros (they do not widen the sparse storage)."""
    g = make()
    gd, _kd = stc.make_generator(g.blocks, g.sizes, g.b)
    want = stc.stc_footprint_bytes(gd, stc.make_options(format=fmt))
    for kw in ({}, {"explicit_zeros": 40}):
        gc, _kc = _csr_gen(g, **kw)
        assert stc.stc_footprint_bytes(gc, stc.make_options(format=fmt)) == want, kw


def _setup_error(gen):
    opt = stc.make_options()
    opt.arena, opt.arena_bytes = 4096, 1 << 40    # never touched: validation fails first
    with pytest.raises(stc.StcError) as e:
        stc.stc_setup(gen, opt)
    return e.value


def test_csr_input_rejections(lib):
    g = synth.qbd(12, 8, 21)
    ip, ix, v = g.to_csr()
    # an entry joining levels 0 and 2 of a QBD (b = 1)
    ix2 = ix.copy()
    ix2[0] = g.offsets[2] + 1
    err = _setup_error(stc.make_generator_csr(ip, ix2, v, g.sizes, 1)[0])
    assert err.status == stc.STC_EINVAL and "outside the block band" in str(err), str(err)
    # a column out of range
    ix2 = ix.copy()
    ix2[5] = g.N + 3
    err = _setup_error(stc.make_generator_csr(ip, ix2, v, g.sizes, 1)[0])
    assert err.status == stc.STC_EINVAL and "outside 0.." in str(err), str(err)
    # a column repeated within a row
    ix2 = ix.copy()
    ix2[ip[3] + 1] = ix2[ip[3]]
    err = _setup_error(stc.make_generator_csr(ip, ix2, v, g.sizes, 1)[0])
    assert err.status == stc.STC_EINVAL and "repeats column" in str(err), str(err)
    # falling row pointers: setup rejects, the sparse footprint is 0
    ip2 = ip.copy()
    ip2[4] = ip2[3] - 1
    gen = stc.make_generator_csr(ip2, ix, v, g.sizes, 1)[0]
    assert stc.stc_footprint_bytes(gen, stc.make_options(format="sparse")) == 0
    err = _setup_error(gen)
    assert err.status == stc.STC_EINVAL and "row pointers" in str(err), str(err)
    # both inputs at once
    gen, _k = stc.make_generator(g.blocks, g.sizes, 1)
    gen.csr_rowptr, gen.csr_col, gen.csr_val = ip.ctypes.data, ix.ctypes.data, v.ctypes.data
    assert stc.stc_footprint_bytes(gen, stc.make_options()) == 0
    assert _setup_error(gen).status == stc.STC_EINVAL
    # a negative rate still reads as "not a generator"
    v2 = v.copy()
    v2[np.flatnonzero(ix != np.repeat(np.arange(g.N), np.diff(ip)))[7]] = -0.5
    err = _setup_error(stc.make_generator_csr(ip, ix, v2, g.sizes, 1)[0])
    assert err.status == stc.STC_ENOTGEN, str(err)
    # without diagonal entries the rows do not sum to 0 unless recomputed
    ip3, ix3, v3 = g.to_csr(drop_diagonal=True)
    err = _setup_error(stc.make_generator_csr(ip3, ix3, v3, g.sizes, 1)[0])
    assert err.status == stc.STC_ENOTGEN and "sums to" in str(err), str(err)


def test_sizes_checked_before_any_scan(lib):
    """A level size above m is an argument error for the footprint and for
    setup alike (the sparse footprint scans the blocks by level size)."""
    g = synth.banded(8, 16, 3, b=2, density=0.3)
    sizes = g.sizes.copy()
    sizes[3] = 40
    gen, _k = stc.make_generator(g.blocks, sizes, 2)
    assert stc.stc_footprint_bytes(gen, stc.make_options(format="sparse")) == 0
    err = _setup_error(gen)
    assert err.status == stc.STC_EINVAL and "sizes[3] = 40" in str(err), str(err)


# --- generators of any block pattern ---------------------------------------

def _gen_csr(g, **kw):
    return stc.make_generator_csr(g.indptr, g.indices, g.data, g.sizes, stc.STC_ANY_PATTERN, **kw)


def test_any_pattern_footprint_and_shape_rules(lib):
    g = synth.localized(20, 16, 4, up=2, down=2, jumps=2, ragged=True)
    gen, _k = _gen_csr(g)
    sparse = stc.stc_footprint_bytes(gen, stc.make_options(format="sparse"))
    assert sparse > 0
    # the pattern needs the ELL storage, and CSR input
    assert stc.stc_footprint_bytes(gen, stc.make_options(format="dense")) == 0
    err = _setup_error(gen)
    assert err.status == stc.STC_EINVAL and "STC_SPARSE" in str(err), str(err)
    blocks = np.zeros((g.L, 1, g.m, g.m))
    gb, _kb = stc.make_generator(blocks, g.sizes, 0)
    gb.b = stc.STC_ANY_PATTERN
    assert stc.stc_footprint_bytes(gb, stc.make_options(format="sparse")) == 0
    # FP32 copies add to the footprint; more far entries add slots
    assert stc.stc_footprint_bytes(gen, stc.make_options(format="sparse", precision="mixed")) > sparse
    g2 = synth.localized(20, 16, 4, up=2, down=2, jumps=6, ragged=True)
    gen2, _k2 = _gen_csr(g2)
    assert stc.stc_footprint_bytes(gen2, stc.make_options(format="sparse")) > sparse


def test_any_pattern_footprint_counts_the_ell_slots(lib):
    """The footprint grows by exactly the ELL slots (12 bytes each in FP64)
    when one column of a level gets one more far entry than any other."""
    g = synth.localized(6, 8, 1, up=1, down=1, jumps=0, backbone=0.1)
    gen, _k = _gen_csr(g)
    base = stc.stc_footprint_bytes(gen, stc.make_options(format="sparse"))
    # add 5 far rates into column 0 of level 4 (rows of level 0 and 1): the
    # far width of level 4 becomes 8 (two quads) from 0
    Q = g.to_scipy().tolil()
    for r in range(5):
        Q[r if r < 3 else 8 + r, 4 * 8] = 0.01
    Q = Q.tocsr()
    Q.setdiag(0.0)
    Q.setdiag(-np.asarray(Q.sum(axis=1)).ravel())
    Q.sort_indices()
    gen2, _k2 = stc.make_generator_csr(Q.indptr, Q.indices, Q.data, g.sizes, stc.STC_ANY_PATTERN)
    grown = stc.stc_footprint_bytes(gen2, stc.make_options(format="sparse"))
    slots = 8 * 8
    assert 0 < grown - base <= slots * 12 + 3 * 256
    assert grown - base >= slots * 12


def test_any_pattern_csr_rejections(lib):
    g = synth.localized(10, 8, 2, up=2, down=1, jumps=2)
    ip, ix, v = g.indptr, g.indices, g.data

    def err_of(ip_, ix_, v_, **kw):
        gen = stc.make_generator_csr(ip_, ix_, v_, g.sizes, stc.STC_ANY_PATTERN, **kw)[0]
        e = stc.StcError
        opt = stc.make_options(format="sparse")
        opt.arena, opt.arena_bytes = 4096, 1 << 40
        import pytest as _p
        with _p.raises(e) as info:
            stc.stc_setup(gen, opt)
        return info.value

    ix2 = ix.copy()
    ix2[5] = g.N + 3
    err = err_of(ip, ix2, v)
    assert err.status == stc.STC_EINVAL and "outside 0.." in str(err), str(err)
    ix2 = ix.copy()
    ix2[ip[3] + 1] = ix2[ip[3]]
    err = err_of(ip, ix2, v)
    assert err.status == stc.STC_EINVAL and "repeats column" in str(err), str(err)
    v2 = v.copy()
    v2[np.flatnonzero(ix != np.repeat(np.arange(g.N), np.diff(ip)))[7]] = -0.5
    err = err_of(ip, ix, v2)
    assert err.status == stc.STC_ENOTGEN and "is not a rate" in str(err), str(err)
    v3 = v.copy()
    v3[np.flatnonzero(ix == np.repeat(np.arange(g.N), np.diff(ip)))[4]] += 1.0
    err = err_of(ip, ix, v3)
    assert err.status == stc.STC_ENOTGEN and "sums to" in str(err), str(err)
    ip2 = ip.copy()
    ip2[4] = ip2[3] - 1
    gen = stc.make_generator_csr(ip2, ix, v, g.sizes, stc.STC_ANY_PATTERN)[0]
    assert stc.stc_footprint_bytes(gen, stc.make_options(format="sparse")) == 0


def test_krylov_workspace_footprint(lib):
    g = synth.qbd(16, 16, 4)
    gen, _k = stc.make_generator(g.blocks, g.sizes, 1)
    base = stc.stc_footprint_bytes(gen, stc.make_options())
    f10 = stc.stc_footprint_bytes(gen, stc.make_options(krylov_restart=10))
    f20 = stc.stc_footprint_bytes(gen, stc.make_options(krylov_restart=20))
    vec = 16 * 16 * 8
    assert f10 - base >= 13 * vec and f20 - f10 >= 10 * vec
    assert stc.stc_footprint_bytes(gen, stc.make_options(krylov_restart=257)) == 0
    assert stc.stc_footprint_bytes(gen, stc.make_options(krylov_restart=-1)) == 0


def test_any_pattern_size_limit_rejected_before_any_scan(lib):
    """L * padded m must stay below 2^31 (32-bit gather indices): 2^24 levels
    of one state padded to 128 is refused by the footprint and by setup,
    before the entries are read."""
    L = 1 << 24
    sizes = np.ones(L, dtype=np.int32)
    indptr = np.zeros(L + 1, dtype=np.int64)
    empty_i = np.zeros(0, dtype=np.int32)
    empty_v = np.zeros(0)
    gen, _k = stc.make_generator_csr(indptr, empty_i, empty_v, sizes, stc.STC_ANY_PATTERN, m=128)
    assert stc.stc_footprint_bytes(gen, stc.make_options(format="sparse")) == 0
    opt = stc.make_options(format="sparse")
    opt.arena, opt.arena_bytes = 4096, 1 << 40
    with pytest.raises(stc.StcError) as e:
        stc.stc_setup(gen, opt)
    assert e.value.status == stc.STC_EINVAL and "2^31" in str(e.value)


def test_prepare_is_host_only_and_checks_the_generator(lib):
    """stc_prepare (the host half of a setup) runs here, with no device: it
    validates and packs; the first bad level is named, as by stc_setup."""
    g = synth.qbd(9, 6, 11, last=4)
    p = stc.Prepared(g.blocks, g.sizes, g.b, precision="mixed")
    assert p.p and p.N == int(np.sum(g.sizes))
    assert p.footprint == stc.stc_footprint_bytes(*_gen_opt(g, precision="mixed")[:2])
    p.close()
    p.close()                       # a second release is a no-op
    bad = g.blocks.copy()
    bad[5, 2, 1, 2] = -0.25         # level 5's up-rate row 1 -> not a generator
    with pytest.raises(stc.StcError) as e:
        stc.Prepared(bad, g.sizes, g.b)
    assert e.value.status == stc.STC_ENOTGEN and "level 5" in str(e.value)
    bad = g.blocks.copy()
    bad[2, 1, 0, 0] += 1.0          # row 0 of level 2 no longer sums to 0
    with pytest.raises(stc.StcError) as e:
        stc.Prepared(bad, g.sizes, g.b)
    assert e.value.status == stc.STC_ENOTGEN and "level 2" in str(e.value)


def test_prepare_takes_dense_banded_storage_only(lib):
    g = synth.qbd(6, 4, 12)
    gen, opt, keep = _gen_opt(g, format="sparse")
    with pytest.raises(stc.StcError) as e:
        stc.stc_prepare(gen, opt)
    assert e.value.status == stc.STC_EINVAL and "dense" in str(e.value)


def test_setup_prepared_rejects_small_arena_before_touching_the_device(lib):
    g = synth.qbd(6, 4, 13)
    p = stc.Prepared(g.blocks, g.sizes, g.b)
    opt = stc.make_options("fp64")
    opt.arena, opt.arena_bytes = 4096, 16
    with pytest.raises(stc.StcError) as e:
        stc.stc_setup_prepared(p.p, opt)
    assert e.value.status == stc.STC_ENOMEM
    opt = stc.make_options("fp64", format="sparse")
    opt.arena, opt.arena_bytes = 4096, 1 << 30
    with pytest.raises(stc.StcError) as e:
        stc.stc_setup_prepared(p.p, opt)
    assert e.value.status == stc.STC_EINVAL
    p.close()


def test_large_blocks_only_for_any_pattern(lib):
    """Blocks above 128 (up to 2048) are taken by generators of any block
    pattern only; the banded kernels stop at 128.  Blocks above 256 pad to
    512, 1024 or 2048, with one partial slot per column slice of a level."""
    g = synth.qbd(4, 4, 2)
    gen, opt, _ = _gen_opt(g)
    gen.m = 200
    assert stc.stc_footprint_bytes(gen, opt) == 0
    import scipy.sparse as sp
    N, m = 600, 256
    Q = sp.random(N, N, density=0.01, random_state=3, format="csr")
    Q.setdiag(0.0)
    Q.setdiag(-np.asarray(Q.sum(axis=1)).ravel())
    Q = Q.tocsr()
    Q.sort_indices()
    sizes = np.array([256, 256, 88], dtype=np.int32)
    gen, keep = stc.make_generator_csr(Q.indptr, Q.indices, Q.data, sizes, stc.STC_ANY_PATTERN, m,
                                       False)
    opt = stc.make_options("fp64", format="sparse")
    fp = stc.stc_footprint_bytes(gen, opt)
    assert fp >= 3 * m * m * 8          # the three 256 x 256 inverses
    for m_big, mp in ((257, 512), (1000, 1024), (2048, 2048)):
        gen.m = m_big
        fp_big = stc.stc_footprint_bytes(gen, opt)
        # inverses and diagonal blocks, FP64, padded to mp
        assert fp_big >= 2 * 3 * mp * mp * 8, m_big
    gen.m = 2049
    assert stc.stc_footprint_bytes(gen, opt) == 0


def test_jgs_footprints_on_any_pattern(lib):
    """Algorithm 1 takes generators of any block pattern at every block size
    up to 2048.  Up to 256 it needs nothing beyond the stair splitting's
    footprint; on the large blocks it adds the split apply's row-range parts,
    8 vectors of L MP FP64 (within the arena's alignment).  jgs_chunks must lie
    in 1..L, and no Krylov workspace is taken."""
    import scipy.sparse as sp
    N = 600
    Q = sp.random(N, N, density=0.01, random_state=4, format="csr")
    Q.setdiag(0.0)
    Q.setdiag(-np.asarray(Q.sum(axis=1)).ravel())
    Q = Q.tocsr()
    Q.sort_indices()
    sizes = np.array([256, 256, 88], dtype=np.int32)
    gen, keep = stc.make_generator_csr(Q.indptr, Q.indices, Q.data, sizes, stc.STC_ANY_PATTERN, 256,
                                       False)
    stair = stc.make_options("fp64", format="sparse")
    jgs = stc.make_options("fp64", format="sparse", method="jgs", jgs_chunks=2)
    assert stc.stc_footprint_bytes(gen, jgs) == stc.stc_footprint_bytes(gen, stair) > 0
    for m_big, mp in ((257, 512), (1000, 1024), (2048, 2048)):
        gen.m = m_big
        extra = stc.stc_footprint_bytes(gen, jgs) - stc.stc_footprint_bytes(gen, stair)
        assert 8 * 3 * mp * 8 <= extra <= 8 * 3 * mp * 8 + 4096, m_big
    gen.m = 256
    for bad in (stc.make_options("fp64", format="sparse", method="jgs", jgs_chunks=0),
                stc.make_options("fp64", format="sparse", method="jgs", jgs_chunks=4),
                stc.make_options("fp64", format="sparse", method="jgs", jgs_chunks=2,
                                 krylov_restart=4)):
        assert stc.stc_footprint_bytes(gen, bad) == 0
