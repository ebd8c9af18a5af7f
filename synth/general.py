"""Seeded generators of any block pattern (input construction only).

These are CSR generators whose nonzero blocks are not confined to a band
around the diagonal: the general localized case of section 2, where level i
may exchange probability with any other level.  The states are numbered level
by level, and the levels are consecutive runs of the state order, of equal size
with a smaller last one (the block partition used in section 3).

Workload recipes (stand-ins for the paper's Markov models, whose rates are not
given):
  * ``mutual_exclusion``  the mutual-exclusion model of the fourth test matrix
                 of section 3: n distinguishable processes, each sleeping or
                 using a resource, at most r of them using it at once.  A
                 sleeping process p asks at rate lam_p and enters if fewer
                 than r processes hold the resource (otherwise nothing
                 changes); a user leaves at rate mu_p.  States are ordered by
                 the number of users, then lexicographically by the set of
                 users.  n = 16, r = 12 gives N = 64839 as in the paper.  The
                 rates are seeded draws (the paper does not give them).
  * ``hessenberg_mmatrix``  random singular M-matrices A = Q^T in banded
                 block lower Hessenberg form, the matrices of Example 3 of
                 section 2 (n blocks of size k, scalar lower bandwidth 4k).
  * ``localized``  random generator with blocks at every level distance up to
                 `up` above and `down` below the diagonal, rates scaled by
                 decay^(|d| - 1), a few long jumps to random far levels, and a
                 nearest-neighbour backbone that makes the chain irreducible;
                 ragged level sizes on request.  up = L, down = 1 gives a
                 block upper Hessenberg generator (the shape of the first test
                 matrix of section 3).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import combinations
from math import comb

import numpy as np


def equal_levels(N: int, m: int) -> np.ndarray:
    """Level sizes: m states per level, the remainder in a smaller last level."""
    L = (N + m - 1) // m
    sizes = np.full(L, m, dtype=np.int32)
    sizes[-1] = N - m * (L - 1)
    return sizes


@dataclass
class SparseGenerator:
    """An N x N generator in CSR form with a level partition."""

    indptr: np.ndarray      # int64 [N+1]
    indices: np.ndarray     # int32 [nnz]
    data: np.ndarray        # float64 [nnz]
    sizes: np.ndarray       # int32 [L]
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.sizes.sum())

    @property
    def L(self) -> int:
        return len(self.sizes)

    @property
    def m(self) -> int:
        return int(self.sizes.max())

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    @property
    def offsets(self) -> np.ndarray:
        off = np.zeros(self.L + 1, dtype=np.int64)
        np.cumsum(self.sizes, out=off[1:])
        return off

    @property
    def csr(self):
        return self.indptr, self.indices, self.data

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.N, self.N))

    def level_of(self) -> np.ndarray:
        return np.repeat(np.arange(self.L), self.sizes)

    def block_reach(self) -> int:
        """Largest level distance |level(row) - level(col)| of a nonzero rate."""
        lev = self.level_of()
        rows = np.repeat(np.arange(self.N), np.diff(self.indptr))
        nz = self.data != 0.0
        if not nz.any():
            return 0
        return int(np.abs(lev[rows[nz]] - lev[self.indices[nz]]).max())


def _from_triplets(rows, cols, vals, N: int, sizes, name: str, extra=None) -> SparseGenerator:
    """Assemble off-diagonal rates into CSR with the diagonal that makes every
    row sum to 0 (the generator convention)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    out = np.bincount(rows, weights=vals, minlength=N)
    rows = np.concatenate([rows, np.arange(N)])
    cols = np.concatenate([cols, np.arange(N)])
    vals = np.concatenate([vals, -out])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    # merge repeated (row, col) pairs
    keep = np.ones(len(rows), dtype=bool)
    keep[1:] = (rows[1:] != rows[:-1]) | (cols[1:] != cols[:-1])
    if not keep.all():
        starts = np.flatnonzero(keep)
        vals = np.add.reduceat(vals, starts)
        rows, cols = rows[starts], cols[starts]
    indptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=indptr[1:])
    return SparseGenerator(indptr, cols.astype(np.int32), vals, np.asarray(sizes, dtype=np.int32),
                           name, extra or {})


def mutual_exclusion_states(n: int, r: int):
    """States (sets of users as bit masks) in the model's order: by the number
    of users, then lexicographically; returns (masks, index of each mask)."""
    masks = []
    for k in range(r + 1):
        for users in combinations(range(n), k):
            masks.append(sum(1 << p for p in users))
    masks = np.array(masks, dtype=np.int64)
    index = {int(s): i for i, s in enumerate(masks)}
    return masks, index


def mutual_exclusion(n: int = 16, r: int = 12, seed: int = 0, *, m: int = 128,
                     lam_range=(0.2, 1.0), mu_range=(0.5, 1.5)) -> SparseGenerator:
    """The mutual-exclusion generator (see the module notes).  extra holds
    the rates lam, mu and the state masks."""
    rng = np.random.default_rng(seed)
    lam = rng.uniform(*lam_range, size=n)
    mu = rng.uniform(*mu_range, size=n)
    masks, index = mutual_exclusion_states(n, r)
    N = len(masks)
    assert N == sum(comb(n, k) for k in range(r + 1))
    rows, cols, vals = [], [], []
    for s, u in enumerate(masks.tolist()):
        users = bin(u).count("1")
        for p in range(n):
            bit = 1 << p
            if u & bit:
                rows.append(s); cols.append(index[u ^ bit]); vals.append(mu[p])
            elif users < r:
                rows.append(s); cols.append(index[u | bit]); vals.append(lam[p])
    return _from_triplets(rows, cols, vals, N, equal_levels(N, m), f"mutex_n{n}_r{r}_m{m}",
                          {"lam": lam, "mu": mu, "masks": masks, "n": n, "r": r})


def mutual_exclusion_pi(g: SparseGenerator) -> np.ndarray:
    """The model's known stationary vector: pi(S) proportional to the product
    of lam_p / mu_p over the users p in S.  Each process alone is a reversible
    two-state chain; blocking the requests that would exceed r users truncates
    the product chain to a subset of its states, which keeps the product form
    restricted to that subset (Kelly's truncation of reversible chains)."""
    rho = g.extra["lam"] / g.extra["mu"]
    masks = g.extra["masks"]
    logw = np.zeros(len(masks))
    for p in range(g.extra["n"]):
        logw += np.where((masks >> p) & 1, np.log(rho[p]), 0.0)
    w = np.exp(logw - logw.max())
    return w / w.sum()


def hessenberg_mmatrix(n: int = 16, k: int = 64, seed: int = 0, *, lower: int = 4,
                       m: int | None = None) -> SparseGenerator:
    """A random singular M-matrix A = Q^T of Example 3: n x n blocks of size
    k, banded block lower Hessenberg.  A_{ij} (i != j) is drawn U[0, 1] inside
    the profile: j in a block column at most one above i's (block
    Hessenberg) and i - j <= lower * k (the scalar lower bandwidth); zero
    outside.  The diagonal makes every column of A, i.e. every row of the
    generator Q, sum to 0.  Levels: equal runs of m states (default k)."""
    rng = np.random.default_rng(seed)
    N = n * k
    i = np.repeat(np.arange(N), N)
    j = np.tile(np.arange(N), N)
    keep = (j // k <= i // k + 1) & (i - j <= lower * k) & (i != j)
    i, j = i[keep], j[keep]
    a = rng.random(len(i))
    # Q_{j,i} = A_{i,j}
    return _from_triplets(j, i, a, N, equal_levels(N, m or k), f"hessenberg_n{n}_k{k}",
                          {"n": n, "k": k, "lower": lower})


def with_levels(g: SparseGenerator, m: int) -> SparseGenerator:
    """The same generator partitioned into equal levels of m states."""
    return SparseGenerator(g.indptr, g.indices, g.data, equal_levels(g.N, m),
                           f"{g.name}_m{m}", dict(g.extra))


def localized(L: int, m: int, seed: int, *, up: int = 3, down: int = 3, density: float = 0.2,
              decay: float = 0.5, jumps: int = 2, ragged: bool = False,
              backbone: float = 0.05) -> SparseGenerator:
    """Random generator with nonzero blocks at level distances 1..up above and
    1..down below the diagonal, `jumps` extra blocks per level at random far
    levels, and a backbone s <-> s+1 of rate `backbone` (irreducibility)."""
    rng = np.random.default_rng(seed)
    if ragged:
        sizes = rng.integers(max(1, m // 2), m + 1, size=L).astype(np.int32)
        sizes[0] = m
    else:
        sizes = np.full(L, m, dtype=np.int32)
    off = np.zeros(L + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    N = int(off[-1])
    rows, cols, vals = [], [], []

    def block(i, k, scale):
        mask = rng.random((sizes[i], sizes[k])) < density
        if i == k:
            np.fill_diagonal(mask, False)
        r, c = np.nonzero(mask)
        rows.append(r + off[i])
        cols.append(c + off[k])
        vals.append(rng.uniform(0.0, scale, size=len(r)))

    for i in range(L):
        block(i, i, 1.0)
        for d in range(1, up + 1):
            if i + d < L:
                block(i, i + d, decay ** (d - 1))
        for d in range(1, down + 1):
            if i - d >= 0:
                block(i, i - d, decay ** (d - 1))
        for _ in range(jumps):
            k = int(rng.integers(L))
            if abs(k - i) > max(up, down):
                block(i, k, decay ** 3)
    s = np.arange(N - 1)
    rows += [s, s + 1]
    cols += [s + 1, s]
    vals += [np.full(N - 1, backbone), np.full(N - 1, backbone)]
    return _from_triplets(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), N,
                          sizes, f"localized_L{L}_m{m}_up{up}_down{down}",
                          {"up": up, "down": down})


def banded_random(N: int, lower: int, upper: int, seed: int, *, per_row: int = 6,
                  m: int = 2048, symmetric: bool = False, backbone: float = 0.05,
                  name: str = "banded_random") -> SparseGenerator:
    """A sparse generator inside a scalar band: each state s gets `per_row`
    transitions to states drawn uniformly from s - lower .. s + upper (s
    excluded), rates U[0, 1], and a backbone s <-> s + 1 of rate `backbone`.
    symmetric: every drawn pair (s, t), t > s, within `upper` (= `lower`)
    gets the same rate both ways, so Q is symmetric, its columns sum to 0 too,
    and the stationary vector is uniform.  Levels: equal runs of m states.
    (Shape stand-ins for the second and third test matrices of section 3: the
    time-sharing model, symmetric with bandwidth 1135, and the priority model,
    lower and upper bandwidths 2370 and 1585; their rates are not given.)"""
    rng = np.random.default_rng(seed)
    s = np.repeat(np.arange(N, dtype=np.int64), per_row)
    if symmetric:
        if lower != upper:
            raise ValueError("a symmetric band has lower == upper")
        t = s + rng.integers(1, upper + 1, size=len(s))
        keep = t < N
        s, t = s[keep], t[keep]
        v = rng.uniform(0.0, 1.0, size=len(s))
        b = np.arange(N - 1)
        rows = np.concatenate([s, t, b, b + 1])
        cols = np.concatenate([t, s, b + 1, b])
        vals = np.concatenate([v, v, np.full(N - 1, backbone), np.full(N - 1, backbone)])
    else:
        d = rng.integers(-lower, upper, size=len(s))
        d = np.where(d >= 0, d + 1, d)            # s itself excluded
        t = s + d
        keep = (t >= 0) & (t < N)
        s, t = s[keep], t[keep]
        v = rng.uniform(0.0, 1.0, size=len(s))
        b = np.arange(N - 1)
        rows = np.concatenate([s, b, b + 1])
        cols = np.concatenate([t, b + 1, b])
        vals = np.concatenate([v, np.full(N - 1, backbone), np.full(N - 1, backbone)])
    return _from_triplets(rows, cols, vals, N, equal_levels(N, m), f"{name}_N{N}_m{m}",
                          {"lower": lower, "upper": upper, "symmetric": symmetric})


def upper_hessenberg(N: int, k: int, seed: int, *, up: int = 4, down: int = 2,
                     mean_jump: float = 2.0, m: int = 512) -> SparseGenerator:
    """A generator that is block upper Hessenberg in levels of k states: each
    state s gets `up` upward transitions, J levels of k states up plus a
    uniform offset inside that level, with J >= 1 geometric of mean
    `mean_jump` (batch arrivals: unbounded jumps up, mostly short), and `down`
    transitions to states at most k below (one level down at a time).  Rates
    U[0, 1].  Levels of the partition: equal runs of m states.  (A shape
    stand-in for the first test matrix of section 3, the retrial queue with
    800 levels of 138 states; its rates are not given.)"""
    rng = np.random.default_rng(seed)
    su = np.repeat(np.arange(N, dtype=np.int64), up)
    J = rng.geometric(1.0 / mean_jump, size=len(su))
    tu = su + J * k + rng.integers(0, k, size=len(su)) - (su % k)
    ku = tu < N
    sd = np.repeat(np.arange(N, dtype=np.int64), down)
    td = sd - rng.integers(1, k + 1, size=len(sd))
    kd = td >= 0
    rows = np.concatenate([su[ku], sd[kd]])
    cols = np.concatenate([tu[ku], td[kd]])
    vals = rng.uniform(0.0, 1.0, size=len(rows))
    return _from_triplets(rows, cols, vals, N, equal_levels(N, m), f"upper_hessenberg_N{N}_m{m}",
                          {"k": k, "up": up, "down": down})
