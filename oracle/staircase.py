"""Algorithm 2 (block staircase splitting, STAIR1 / STAIR2) and Algorithm 1
(the [BB] composite block Jacobi / block Gauss-Seidel scheme, "JGS"), FP64.

Both implement the normalised power-type scheme of section 2, eq. (mainsch):
M x^(k+1) = N x^(k), then x^(k+1) <- x^(k+1) / e^T x^(k+1), for a regular
splitting Q^T = M - N.  Notation follows section 2: A = Q^T is split into
blocks A_{i,k} = (Q^T)_{i,k} = (Q_{k,i})^T, i, k over the L levels.

Stair matrices (section 2): in the type-1 stair matrix M1 the odd block rows
(1-based) keep only A_{i,i} while the even block rows keep A_{i,i-1}, A_{i,i},
A_{i,i+1}; type 2 swaps the parities.  Solving M x = r therefore takes two
parallel steps: the diagonal-only rows first ("phase A"), then the stair rows
from the fresh neighbours ("phase B").  With 0-based levels, phase A of type 1
is the even levels and phase A of type 2 the odd levels.

Readings where the printed algorithm is ambiguous:
  * The first parallel loop of Algorithm 2 gathers, for every level i, the
    blocks that are NOT in the stair row, i.e. k outside J_i and k != i
    (J_i = {i-1, i+1} on stair rows, {i} on diagonal-only rows).  Taking the
    printed index set literally would also subtract A_{i,i} x_i, and pi would
    not be a fixed point of the scheme.
  * The loop guard is "err > tol and it < maxit", with err = +inf before the
    first sweep (the printed guard has the comparison reversed; the stopping
    test of section 3 stops once ||x^(k) - x^(k+1)||_1 <= eps or k >= maxit).
  * eps is positive (section 3 prints a negative value, read as 1e-9).
  * The change err is measured after normalisation, against the previous
    normalised iterate.
  * Blocks A_{i,i}^{-1} are applied by an LU solve of each diagonal block.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .dense import level_offsets, residual_1

STOP_DIFF = "diff"          # ||x^(k+1) - x^(k)||_1 <= tol   (section 3)
STOP_RESIDUAL = "residual"  # ||Q^T x^(k+1)||_1 <= tol


class DegenerateIterate(ArithmeticError):
    """e^T z <= 0 (or not finite): the sweep produced no mass to normalise."""


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    err: float
    residual: float
    converged: bool
    history: list = field(default_factory=list)


class BlockSystem:
    """Block view of A = Q^T for a block-banded generator (b = block bandwidth)."""

    def __init__(self, blocks: np.ndarray, sizes, b: int):
        self.blocks = blocks
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.b = int(b)
        self.L = blocks.shape[0]
        self.off = level_offsets(self.sizes)
        self.N = int(self.off[-1])

    def A(self, i: int, k: int) -> np.ndarray:
        """Block A_{i,k} = (Q_{k,i})^T of A = Q^T (zero outside the band)."""
        d = i - k  # Q_{k,i} sits in row-level k at slot (i - k) + b
        if abs(d) > self.b or not (0 <= k < self.L):
            return np.zeros((self.sizes[i], self.sizes[k]))
        return self.blocks[k, d + self.b, : self.sizes[k], : self.sizes[i]].T

    def seg(self, x: np.ndarray, i: int) -> np.ndarray:
        return x[self.off[i]: self.off[i + 1]]

    def band(self, i: int):
        return range(max(0, i - self.b), min(self.L, i + self.b + 1))

    def residual(self, x: np.ndarray) -> float:
        return residual_1(self.blocks, self.sizes, self.b, x)


class SparseBlockSystem:
    """Block view of A = Q^T for a generator of any block pattern (the general
    localized case of section 2: level i may couple to any level k).

    Q is given as an N x N scipy.sparse matrix, states numbered level by level
    with the given level sizes.  Only the nonzero blocks are kept, densified:
    band(i) lists the levels k (i included) whose block A_{i,k} is nonzero, so
    the sweep below visits exactly the blocks the first loop of Algorithm 2
    sums over."""

    def __init__(self, Q, sizes):
        import scipy.sparse as sp
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.L = len(self.sizes)
        self.off = level_offsets(self.sizes)
        self.N = int(self.off[-1])
        self.Q = sp.csr_matrix(Q)
        if self.Q.shape != (self.N, self.N):
            raise ValueError("Q must be N x N with N = sum of the level sizes")
        At = self.Q.T.tocsr()   # A = Q^T
        lev = np.repeat(np.arange(self.L), self.sizes)
        self.blocks = {}
        self.nbr = []
        for i in range(self.L):
            rows = At[self.off[i]: self.off[i + 1]]
            ks = sorted(set(lev[rows.indices].tolist()) | {i})
            for k in ks:
                self.blocks[(i, k)] = rows[:, self.off[k]: self.off[k + 1]].toarray()
            self.nbr.append(ks)

    def A(self, i: int, k: int) -> np.ndarray:
        blk = self.blocks.get((i, k))
        if blk is None:
            return np.zeros((self.sizes[i], self.sizes[k]))
        return blk

    def seg(self, x: np.ndarray, i: int) -> np.ndarray:
        return x[self.off[i]: self.off[i + 1]]

    def band(self, i: int):
        return self.nbr[i]

    def residual(self, x: np.ndarray) -> float:
        """||Q^T x||_1 (eq. (1)), by one sparse product."""
        return float(np.abs(self.Q.T @ x).sum())


def phase_sets(L: int, stair_type: int):
    """(diagonal-only levels, stair levels), 0-based, for stair type 1 or 2."""
    if stair_type not in (1, 2):
        raise ValueError("stair_type must be 1 or 2")
    first = 0 if stair_type == 1 else 1
    diag_only = [i for i in range(L) if i % 2 == first % 2]
    stair = [i for i in range(L) if i % 2 != first % 2]
    return diag_only, stair


def J_set(i: int, L: int, stair_type: int):
    """J_i of Algorithm 2 (0-based): {i-1, i+1} on stair rows, {i} otherwise."""
    _, stair = phase_sets(L, stair_type)
    if i in stair:
        return [k for k in (i - 1, i + 1) if 0 <= k < L]
    return [i]


def staircase_sweep(sys: BlockSystem, x: np.ndarray, stair_type: int = 1,
                    literal_J: bool = False):
    """One sweep of Algorithm 2 from the normalised iterate x.

    Returns (z, err) with z normalised (e^T z = 1) and err = ||z - x||_1.
    ``literal_J`` reproduces the printed first loop (sum over k not in J_i,
    which includes k = i on stair rows); it exists only so that a test can
    show that this reading does not have pi as a fixed point.
    """
    z = stair_apply(sys, x, stair_type, literal_J)
    s = z.sum()
    if not (np.isfinite(s) and s > 0.0):
        raise DegenerateIterate(f"e^T z = {s}")
    z /= s
    return z, float(np.abs(z - x).sum())


def stair_apply(sys, x: np.ndarray, stair_type: int = 1, literal_J: bool = False) -> np.ndarray:
    """z = M^{-1} N x for the stair splitting Q^T = M - N, by the three
    parallel loops of Algorithm 2 without the normalisation (any real x)."""
    L = sys.L
    diag_only, stair = phase_sets(L, stair_type)
    Js = {i: J_set(i, L, stair_type) for i in range(L)}
    z = np.zeros(sys.N)
    # first parallel loop: gather the blocks outside the stair row (old x)
    for i in range(L):
        skip = set(Js[i]) if literal_J else set(Js[i]) | {i}
        acc = np.zeros(sys.sizes[i])
        for k in sys.band(i):
            if k not in skip:
                acc -= sys.A(i, k) @ sys.seg(x, k)
        sys.seg(z, i)[:] = acc
    # second parallel loop: diagonal-only rows
    for i in diag_only:
        sys.seg(z, i)[:] = np.linalg.solve(sys.A(i, i), sys.seg(z, i))
    # third parallel loop: stair rows, from the fresh neighbours
    for i in stair:
        rhs = sys.seg(z, i).copy()
        for k in Js[i]:
            rhs -= sys.A(i, k) @ sys.seg(z, k)
        sys.seg(z, i)[:] = np.linalg.solve(sys.A(i, i), rhs)
    return z


def staircase_solve(blocks: np.ndarray, sizes, b: int, *, stair_type: int = 1,
                    x0: np.ndarray | None = None, tol: float = 1e-9,
                    maxit: int = 10_000, stop: str = STOP_DIFF,
                    keep_history: bool = False) -> SolveResult:
    """Algorithm 2: repeat sweeps until the stop quantity is <= tol or maxit
    sweeps were done.  Default start e/N; the start is normalised first."""
    return solve_system(BlockSystem(blocks, sizes, b), stair_type=stair_type, x0=x0, tol=tol,
                        maxit=maxit, stop=stop, keep_history=keep_history)


def solve_system(sys, *, stair_type: int = 1, x0: np.ndarray | None = None, tol: float = 1e-9,
                 maxit: int = 10_000, stop: str = STOP_DIFF,
                 keep_history: bool = False) -> SolveResult:
    """Algorithm 2 on a block system (BlockSystem or SparseBlockSystem)."""
    x = np.full(sys.N, 1.0 / sys.N) if x0 is None else np.asarray(x0, float) / np.sum(x0)
    it, err = 0, np.inf
    hist = []
    while err > tol and it < maxit:
        z, diff = staircase_sweep(sys, x, stair_type)
        err = diff if stop == STOP_DIFF else sys.residual(z)
        if keep_history:
            hist.append(err)
        x = z
        it += 1
    res = sys.residual(x)
    return SolveResult(x, it, float(err), res, bool(err <= tol), hist)


def jgs_sweep(sys: BlockSystem, x: np.ndarray, chunks):
    """One sweep of Algorithm 1: block Jacobi across the chunks (processors),
    block Gauss-Seidel inside each chunk.  ``chunks`` lists (start, count) of
    consecutive levels covering 0..L-1.  Returns (z, err) as above."""
    z = np.zeros(sys.N)
    for start, count in chunks:
        for k in range(start, start + count):
            acc = np.zeros(sys.sizes[k])
            for s in sys.band(k):
                if s == k:
                    continue
                v = sys.seg(z, s) if start <= s < k else sys.seg(x, s)
                acc += sys.A(k, s) @ v
            sys.seg(z, k)[:] = -np.linalg.solve(sys.A(k, k), acc)
    s = z.sum()
    if not (np.isfinite(s) and s > 0.0):
        raise DegenerateIterate(f"e^T z = {s}")
    z /= s
    return z, float(np.abs(z - x).sum())
