"""Sampled outputs of one stair sweep from windows of levels (test helper).

With block bandwidth 1 the sweep of Algorithm 2 is local: phase A of level i
reads the previous iterate at i - 1 and i + 1, and phase B of level i reads
phase A at i - 1 and i + 1.  The oracle's stair_apply over the levels
[lo, hi) alone, with lo even so that the phases keep their parity, therefore
gives the exact unnormalised values of levels lo + 2 .. hi - 3, and at the
chain's own ends of levels 0 .. and .. L - 1."""
import numpy as np

from oracle import staircase


def windows(L, width=12, count=24):
    """Even window starts spread over the chain, both ends included."""
    starts = np.linspace(0, max(L - width, 0), count).astype(int) // 2 * 2
    return sorted(set(int(s) for s in starts) | {0, max(L - width, 0) // 2 * 2})


def sampled_stair_apply(g, x, width=12, count=24):
    """(indices, values): exact entries of M^{-1} N x (stair type 1) for the
    interior levels of each window of a block-tridiagonal generator."""
    if g.b != 1:
        raise ValueError("windows are exact for block bandwidth 1 only")
    off = np.concatenate([[0], np.cumsum(g.sizes)])
    idx, vals = [], []
    for lo in windows(g.L, width, count):
        hi = g.L if lo + width + 1 >= g.L else lo + width   # the last window reaches L
        sys_w = staircase.BlockSystem(g.blocks[lo:hi], g.sizes[lo:hi], g.b)
        u = staircase.stair_apply(sys_w, x[off[lo]:off[hi]], 1)
        first = lo if lo == 0 else lo + 2
        last = hi - 1 if hi == g.L else hi - 3
        if last < first:
            continue
        idx.append(np.arange(off[first], off[last + 1]))
        vals.append(u[off[first] - off[lo]:off[last + 1] - off[lo]])
    return np.concatenate(idx), np.concatenate(vals)
