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
