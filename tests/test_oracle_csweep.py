"""Pins of the C/OpenMP oracle sweep (used for the CPU baseline)."""
import os

import numpy as np
import pytest

import synth
from oracle import csweep, dense, gth, splittings

pytestmark = pytest.mark.skipif(not os.path.exists(csweep.LIB),
                                reason="oracle/_csweep.so not built")


@pytest.mark.parametrize("b,stair_type,last", [(1, 1, None), (1, 2, 3), (2, 1, 2), (2, 2, None)])
def test_csweep_equals_dense_splitting(b, stair_type, last):
    if b == 1:
        g = synth.qbd(9, 5, 80 + stair_type, last=last)
    else:
        g = synth.banded(9, 5, 82 + stair_type, b=2, density=0.5, last=last)
    A = dense.assemble_A(g.blocks, g.sizes, g.b)
    T = splittings.iteration_matrix(A, g.sizes, f"stair{stair_type}")
    x = synth.positive_start(g, 4)
    want = T @ x
    want /= want.sum()
    cs = csweep.CSweep(g.blocks, g.sizes, g.b, stair_type, threads=2)
    z = np.zeros((g.L, g.m))
    err = cs.sweep(g.pack(x), z)
    assert np.abs(g.unpack(z) - want).sum() < 1e-14
    assert abs(err - np.abs(want - x).sum()) < 1e-14
    assert np.all(z[-1, g.sizes[-1]:] == 0.0)


def test_csweep_fixed_point():
    g = synth.qbd(12, 6, 85, last=4)
    pi = gth.gth(dense.assemble_Q(g.blocks, g.sizes, g.b))
    cs = csweep.CSweep(g.blocks, g.sizes, g.b, 1, threads=3)
    z = np.zeros((g.L, g.m))
    assert cs.sweep(g.pack(pi), z) < 1e-14


def test_csweep_degenerate_start():
    g = synth.qbd(6, 3, 86)
    x = np.zeros((g.L, g.m))
    x[0] = 1.0 / g.m
    cs = csweep.CSweep(g.blocks, g.sizes, g.b, 1, threads=1)
    with pytest.raises(ArithmeticError):
        cs.sweep(x, np.zeros_like(x))


@pytest.mark.parametrize("stair_type", [1, 2])
@pytest.mark.parametrize("cfg", [dict(L=12, m=6, seed=1, up=2, down=2, jumps=3, ragged=True),
                                 dict(L=16, m=4, seed=2, up=16, down=1, jumps=0)],
                         ids=["ragged_far", "hessenberg"])
def test_general_c_sweep_equals_stair_matrix_definition(cfg, stair_type):
    """The C sweep for generators of any block pattern: one sweep is the
    normalised M^{-1} N x of the dense stair matrix (section 2), and the
    fixed point is the GTH vector."""
    from oracle import gth, splittings
    g = synth.localized(**cfg)
    A = g.to_scipy().T.toarray()
    M = splittings.splitting_M(A, g.sizes, f"stair{stair_type}")
    x = np.random.default_rng(3).uniform(0.5, 1.5, g.N)
    x /= x.sum()
    want = np.linalg.solve(M, (M - A) @ x)
    want /= want.sum()
    c = csweep.CGenSweep(g.to_scipy(), g.sizes, stair_type=stair_type)
    z = np.zeros(g.N)
    err = c.sweep(x, z)
    assert np.abs(z - want).sum() < 1e-13
    assert abs(err - np.abs(want - x).sum()) < 1e-13
    pi = gth.gth(g.to_scipy().toarray())
    z2 = np.zeros(g.N)
    c.sweep(pi.copy(), z2)
    assert np.abs(z2 - pi).sum() < 1e-13
