"""Block GTH: linear level reduction for block-banded generators.

Textbook block elimination of the levels from the last one down (a block form
of GTH state reduction; the paper does not use it).  It gives the reference
stationary vector for chains too large for dense GTH.

For a block-tridiagonal generator (levels 0..L-1), eliminating level i from
the chain censored to levels 0..i gives
    R_i     = Q_{i-1,i} (-S_i)^{-1}
    S_{i-1} = Q_{i-1,i-1} + R_i Q_{i,i-1},          S_{L-1} = Q_{L-1,L-1},
and pi_i = pi_{i-1} R_i, with pi_0 S_0 = 0.  S_i is the level-i block of the
censored generator, so its rows lose exactly the rate of Q_{i,i-1}; its
diagonal is recomputed from that fact as a sum of non-negative terms (the GTH
device), which avoids cancellation.  Level 0 is solved by dense GTH.

A generator of block bandwidth b is first regrouped into super-levels of b
consecutive levels, which makes it block-tridiagonal.
"""
from __future__ import annotations

import numpy as np

from .dense import level_offsets
from .gth import gth


def _super_levels(blocks: np.ndarray, sizes, b: int):
    """Regroup into block-tridiagonal super-levels; returns (diag, up, down)
    lists of dense blocks: diag[s]=Q_{s,s}, up[s]=Q_{s,s+1}, down[s]=Q_{s,s-1}."""
    L = blocks.shape[0]
    groups = [list(range(g, min(L, g + b))) for g in range(0, L, b)]
    off = level_offsets(sizes)

    def gather(rows, cols):
        n_r = sum(int(sizes[i]) for i in rows)
        n_c = sum(int(sizes[k]) for k in cols)
        out = np.zeros((n_r, n_c))
        r0 = 0
        for i in rows:
            c0 = 0
            for k in cols:
                d = k - i
                if abs(d) <= b:
                    out[r0:r0 + sizes[i], c0:c0 + sizes[k]] = \
                        blocks[i, d + b, : sizes[i], : sizes[k]]
                c0 += sizes[k]
            r0 += sizes[i]
        return out

    S = len(groups)
    diag = [gather(groups[s], groups[s]) for s in range(S)]
    up = [gather(groups[s], groups[s + 1]) if s + 1 < S else None for s in range(S)]
    down = [gather(groups[s], groups[s - 1]) if s > 0 else None for s in range(S)]
    del off
    return diag, up, down


def _recompute_diagonal(S: np.ndarray, leak_rows: np.ndarray) -> np.ndarray:
    """diag(S) := -(off-diagonal row sums of S + rate leaving the level set)."""
    S = S.copy()
    n = S.shape[0]
    idx = np.arange(n)
    S[idx, idx] = 0.0
    S[idx, idx] = -(S.sum(axis=1) + leak_rows)
    return S


def level_reduction(blocks: np.ndarray, sizes, b: int) -> np.ndarray:
    """Stationary vector (compact, length N) of a block-banded generator, FP64."""
    diag, up, down = _super_levels(blocks, sizes, b)
    S_count = len(diag)
    R = [None] * S_count
    S_cur = diag[-1]
    for s in range(S_count - 1, 0, -1):
        leak = down[s].sum(axis=1)            # rate from super-level s down to s-1
        S_cur = _recompute_diagonal(S_cur, leak)
        # R_s = Q_{s-1,s} (-S_s)^{-1}   <=>   (-S_s)^T R_s^T = Q_{s-1,s}^T
        R[s] = np.linalg.solve(-S_cur.T, up[s - 1].T).T
        S_cur = diag[s - 1] + R[s] @ down[s]
    S0 = _recompute_diagonal(S_cur, np.zeros(S_cur.shape[0]))
    parts = [gth(S0)]
    for s in range(1, S_count):
        parts.append(parts[-1] @ R[s])
    pi = np.concatenate(parts)
    return pi / pi.sum()
