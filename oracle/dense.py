"""Dense forms of the problem statement (eq. (1), section 1 and section 2).

The stationary vector solves Q^T pi = 0, pi >= 0, e^T pi = 1.  The paper
partitions Q^T into blocks (Q^T)_{i,k} of size n_i x n_k (section 2); with the
generator stored by blocks Q_{i,k}, the block (Q^T)_{i,k} is (Q_{k,i})^T.
"""
from __future__ import annotations

import numpy as np


def level_offsets(sizes) -> np.ndarray:
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def assemble_Q(blocks: np.ndarray, sizes, b: int) -> np.ndarray:
    """Dense N x N generator from padded per-level blocks blocks[i, d+b] = Q_{i,i+d}."""
    L = blocks.shape[0]
    off = level_offsets(sizes)
    N = int(off[-1])
    Q = np.zeros((N, N))
    for i in range(L):
        for d in range(-b, b + 1):
            k = i + d
            if 0 <= k < L:
                Q[off[i]:off[i + 1], off[k]:off[k + 1]] = \
                    blocks[i, d + b, : sizes[i], : sizes[k]]
    return Q


def assemble_A(blocks: np.ndarray, sizes, b: int) -> np.ndarray:
    """A = Q^T, the matrix the splittings of section 2 act on."""
    return assemble_Q(blocks, sizes, b).T.copy()


def residual_1(blocks: np.ndarray, sizes, b: int, x: np.ndarray) -> float:
    """||Q^T x||_1, summed block by block: (Q^T x)_k = sum_i Q_{i,k}^T x_i."""
    L = blocks.shape[0]
    off = level_offsets(sizes)
    total = 0.0
    for k in range(L):
        acc = np.zeros(sizes[k])
        for d in range(-b, b + 1):
            i = k + d
            if 0 <= i < L:
                # block Q_{i,k} sits in row-level i at slot (k - i) + b
                Qik = blocks[i, (k - i) + b, : sizes[i], : sizes[k]]
                acc += Qik.T @ x[off[i]:off[i + 1]]
        total += np.abs(acc).sum()
    return float(total)


def nullspace_solve(Q: np.ndarray) -> np.ndarray:
    """Brute-force pi for a tiny irreducible generator: replace one equation
    of Q^T pi = 0 by e^T pi = 1 and solve the nonsingular system (rank of Q is
    N-1, section 1)."""
    N = Q.shape[0]
    A = Q.T.copy()
    A[-1, :] = 1.0
    rhs = np.zeros(N)
    rhs[-1] = 1.0
    return np.linalg.solve(A, rhs)
