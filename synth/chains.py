"""Seeded block-banded CTMC generators (input construction only).

Convention (problem statement, eq. (1) of the paper): Q is the generator of a
continuous-time chain, off-diagonal entries >= 0 and every row sums to 0; the
stationary vector solves Q^T pi = 0, pi >= 0, e^T pi = 1.  States are grouped
into L levels ("blocks" in the paper's partition of Q^T, section 2); level i
holds n_i states, n_i <= m.

Storage used by every consumer: ``blocks[i, d + b]`` is the generator block
Q_{i, i+d} (rows = states of level i, columns = states of level i+d), row-major,
padded with zeros to m x m.  Slots whose level i+d is outside [0, L) are zero.
The paper works with the blocks of Q^T; the block (Q^T)_{i,k} is the transpose
of Q_{k,i}.

Workload recipes (stand-ins for the paper's Markov models, which are not
reproduced):
  * ``qbd``      level-dependent QBD: up block Q_{i,i+1} ~ Bernoulli(p)*U[0,up_max],
                 down block Q_{i,i-1} ~ Bernoulli(p)*U[0,down_max], dense
                 U[0,1] off-diagonal rates inside a level; a fresh draw per level.
  * ``banded``   block-pentadiagonal (b=2) generator with sparse (10 %) blocks,
                 rates U[0, decay^(|d|-1)] at block distance |d|.
  * ``planted_reversible``  reversible chain with a known stationary vector
                 (detailed balance), used as an exact target.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 230207551


def config_seed(index: int) -> int:
    """Seed of the index-th benchmark workload (recorded in every result)."""
    return BASE_SEED + int(index)


@dataclass
class BlockGenerator:
    """A block-banded generator Q in padded per-level storage."""

    L: int
    m: int
    b: int
    blocks: np.ndarray                      # float64 [L, 2b+1, m, m]
    sizes: np.ndarray = field(default=None)  # int32 [L]; level sizes n_i <= m
    name: str = ""

    def __post_init__(self):
        if self.sizes is None:
            self.sizes = np.full(self.L, self.m, dtype=np.int32)
        self.sizes = np.ascontiguousarray(self.sizes, dtype=np.int32)
        assert self.blocks.shape == (self.L, 2 * self.b + 1, self.m, self.m)
        assert self.blocks.dtype == np.float64

    @property
    def N(self) -> int:
        return int(self.sizes.sum())

    @property
    def offsets(self) -> np.ndarray:
        off = np.zeros(self.L + 1, dtype=np.int64)
        np.cumsum(self.sizes, out=off[1:])
        return off

    def block(self, i: int, k: int) -> np.ndarray:
        """Generator block Q_{i,k} cut to its true shape (n_i x n_k)."""
        d = k - i
        if abs(d) > self.b or not (0 <= k < self.L):
            return np.zeros((self.sizes[i], self.sizes[k]))
        return self.blocks[i, d + self.b, : self.sizes[i], : self.sizes[k]]

    def to_csr(self, drop_diagonal: bool = False, explicit_zeros: int = 0, seed: int = 0):
        """The same generator as one N x N CSR matrix (indptr int64, indices
        int32, data float64), states numbered level by level.  Entries are the
        nonzeros of the blocks; drop_diagonal leaves out Q's diagonal entries;
        explicit_zeros adds that many stored zeros at random in-band positions
        that hold no rate (a storage variant, not a different matrix)."""
        off = self.offsets
        rows, cols, vals = [], [], []
        for i in range(self.L):
            for d in range(-self.b, self.b + 1):
                k = i + d
                if not (0 <= k < self.L):
                    continue
                B = self.block(i, k)
                r, c = np.nonzero(B)
                v = B[r, c]
                if d == 0 and drop_diagonal:
                    keep = r != c
                    r, c, v = r[keep], c[keep], v[keep]
                rows.append(r + off[i])
                cols.append(c + off[k])
                vals.append(v)
        rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
        if explicit_zeros:
            rng = np.random.default_rng(seed)
            taken = set(zip(rows.tolist(), cols.tolist()))
            zr, zc = [], []
            while len(zr) < explicit_zeros:
                i = int(rng.integers(self.L))
                k = int(np.clip(i + rng.integers(-self.b, self.b + 1), 0, self.L - 1))
                r = int(off[i] + rng.integers(self.sizes[i]))
                c = int(off[k] + rng.integers(self.sizes[k]))
                if (r, c) in taken or (drop_diagonal and r == c):
                    continue
                taken.add((r, c))
                zr.append(r)
                zc.append(c)
            rows = np.concatenate([rows, np.array(zr, dtype=rows.dtype)])
            cols = np.concatenate([cols, np.array(zc, dtype=cols.dtype)])
            vals = np.concatenate([vals, np.zeros(len(zr))])
        order = np.lexsort((cols, rows))
        rows, cols, vals = rows[order], cols[order], vals[order]
        indptr = np.zeros(self.N + 1, dtype=np.int64)
        np.cumsum(np.bincount(rows, minlength=self.N), out=indptr[1:])
        return indptr, cols.astype(np.int32), vals.astype(np.float64)

    def pack(self, x: np.ndarray) -> np.ndarray:
        """Compact N-vector -> padded [L, m] array (padding = 0)."""
        out = np.zeros((self.L, self.m), dtype=x.dtype)
        off = self.offsets
        for i in range(self.L):
            out[i, : self.sizes[i]] = x[off[i]: off[i + 1]]
        return out

    def unpack(self, xp: np.ndarray) -> np.ndarray:
        """Padded [L, m] array -> compact N-vector."""
        if np.all(self.sizes == self.m):
            return np.ascontiguousarray(xp.reshape(-1))
        return np.concatenate([xp[i, : self.sizes[i]] for i in range(self.L)])


def _level_mask(sizes: np.ndarray, L: int, m: int, b: int) -> np.ndarray:
    """1 where blocks[i, d+b, r, c] is a real entry (row < n_i, col < n_{i+d})."""
    mask = np.zeros((L, 2 * b + 1, m, m), dtype=bool)
    ar = np.arange(m)
    for d in range(-b, b + 1):
        lo, hi = max(0, -d), min(L, L - d)
        for i in range(lo, hi):
            mask[i, d + b] = (ar[:, None] < sizes[i]) & (ar[None, :] < sizes[i + d])
    return mask


def _set_diagonal(blocks: np.ndarray, sizes: np.ndarray, b: int) -> None:
    """Make every row of Q sum to zero by setting diag(Q_ii) (generator convention)."""
    L, _, m, _ = blocks.shape
    ar = np.arange(m)
    for i in range(L):
        n = sizes[i]
        blocks[i, b, ar, ar] = 0.0
        out = blocks[i].sum(axis=(0, 2))        # row sums of off-diagonal rates
        out[n:] = 0.0
        blocks[i, b, ar, ar] = -out


def _sizes(L: int, m: int, last: int | None) -> np.ndarray:
    sizes = np.full(L, m, dtype=np.int32)
    if last is not None:
        assert 1 <= last <= m
        sizes[-1] = last
    return sizes


def qbd(L: int, m: int, seed: int, *, up_max: float = 0.5, down_max: float = 1.0,
        density: float = 0.3, last: int | None = None, chunk: int = 64,
        name: str = "") -> BlockGenerator:
    """Level-dependent QBD (block-tridiagonal) generator.

    Up block Q_{i,i+1}: Bernoulli(density) x U[0, up_max]; down block
    Q_{i,i-1}: Bernoulli(density) x U[0, down_max]; within-level rates dense
    U[0,1].  Level 0 has no down block and level L-1 no up block.  An up or
    down block that comes out all zero is drawn again so that the chain stays
    irreducible.  ``last`` gives a ragged last level (equal sizes except the
    remainder, as in the paper's experiments, section 3).
    """
    b = 1
    sizes = _sizes(L, m, last)
    rng = np.random.Generator(np.random.PCG64(seed))
    blocks = np.zeros((L, 3, m, m))
    ar = np.arange(m)
    for c0 in range(0, L, chunk):
        c1 = min(L, c0 + chunk)
        n = c1 - c0
        inner = rng.random((n, m, m))
        inner[:, ar, ar] = 0.0
        up = (rng.random((n, m, m)) < density) * rng.random((n, m, m)) * up_max
        down = (rng.random((n, m, m)) < density) * rng.random((n, m, m)) * down_max
        blocks[c0:c1, 1] = inner
        blocks[c0:c1, 2] = up
        blocks[c0:c1, 0] = down
    blocks[0, 0] = 0.0
    blocks[L - 1, 2] = 0.0
    mask = _level_mask(sizes, L, m, b)
    blocks *= mask
    # irreducibility: every present up/down block needs at least one rate
    for i in range(L):
        for slot, hi in ((0, down_max), (2, up_max)):
            if not mask[i, slot].any():
                continue
            while not blocks[i, slot].any():
                draw = (rng.random((m, m)) < density) * rng.random((m, m)) * hi
                blocks[i, slot] = draw * mask[i, slot]
    _set_diagonal(blocks, sizes, b)
    return BlockGenerator(L, m, b, blocks, sizes, name or f"qbd_L{L}_m{m}")


def banded(L: int, m: int, seed: int, *, b: int = 2, density: float = 0.1,
           decay: float = 0.5, inner_density: float | None = None,
           last: int | None = None, chunk: int = 32, name: str = "") -> BlockGenerator:
    """Block-banded (localized) generator with sparse blocks.

    Block Q_{i,i+d}, 1 <= |d| <= b: Bernoulli(density) x U[0, decay^(|d|-1)];
    within-level rates Bernoulli(inner_density or density) x U[0,1].  Blocks at
    distance 1 that come out all zero are drawn again (irreducibility); a level
    whose rows leak nowhere is repaired the same way.
    """
    sizes = _sizes(L, m, last)
    idn = density if inner_density is None else inner_density
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = 2 * b + 1
    blocks = np.zeros((L, nb, m, m))
    ar = np.arange(m)
    for c0 in range(0, L, chunk):
        c1 = min(L, c0 + chunk)
        n = c1 - c0
        for d in range(-b, b + 1):
            if d == 0:
                draw = (rng.random((n, m, m)) < idn) * rng.random((n, m, m))
                draw[:, ar, ar] = 0.0
            else:
                scale = decay ** (abs(d) - 1)
                draw = (rng.random((n, m, m)) < density) * rng.random((n, m, m)) * scale
            blocks[c0:c1, d + b] = draw
    mask = _level_mask(sizes, L, m, b)
    blocks *= mask
    for i in range(L):
        for d in (-1, 1):
            s = d + b
            if not mask[i, s].any():
                continue
            while not blocks[i, s].any():
                draw = (rng.random((m, m)) < density) * rng.random((m, m))
                blocks[i, s] = draw * mask[i, s]
    _set_diagonal(blocks, sizes, b)
    return BlockGenerator(L, m, b, blocks, sizes, name or f"banded_b{b}_L{L}_m{m}")


def skip_free(L: int, m: int, seed: int, *, b: int = 4, up_density: float = 0.3,
              decay: float = 0.5, down_max: float = 1.0, last: int | None = None,
              chunk: int = 32, name: str = "") -> BlockGenerator:
    """Level-dependent generator that is skip-free to the left (M/G/1 type):
    from level i the chain moves down by one level at most, and up by 1..b
    levels with rates that decay with the jump.

    Q_{i,i-1}: Bernoulli(0.3) x U[0, down_max]; Q_{i,i+d}, 1 <= d <= b:
    Bernoulli(up_density) x U[0, decay^(d-1)] / 2; within-level rates dense
    U[0, 1].  The blocks Q_{i,i-d}, d >= 2, are zero.  Stored in the block
    band of width b, so half of the stored off-diagonal slots are empty.
    All-zero blocks at distance 1 are drawn again (irreducibility).
    """
    sizes = _sizes(L, m, last)
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = 2 * b + 1
    blocks = np.zeros((L, nb, m, m))
    ar = np.arange(m)
    for c0 in range(0, L, chunk):
        c1 = min(L, c0 + chunk)
        n = c1 - c0
        inner = rng.random((n, m, m))
        inner[:, ar, ar] = 0.0
        blocks[c0:c1, b] = inner
        blocks[c0:c1, b - 1] = (rng.random((n, m, m)) < 0.3) * rng.random((n, m, m)) * down_max
        for d in range(1, b + 1):
            blocks[c0:c1, b + d] = ((rng.random((n, m, m)) < up_density) *
                                    rng.random((n, m, m)) * 0.5 * decay ** (d - 1))
    mask = _level_mask(sizes, L, m, b)
    blocks *= mask
    for i in range(L):
        for s_, dens, scale in ((b - 1, 0.3, down_max), (b + 1, up_density, 0.5)):
            if not mask[i, s_].any():
                continue
            while not blocks[i, s_].any():
                blocks[i, s_] = (rng.random((m, m)) < dens) * rng.random((m, m)) * scale * mask[i, s_]
    _set_diagonal(blocks, sizes, b)
    return BlockGenerator(L, m, b, blocks, sizes, name or f"skipfree_b{b}_L{L}_m{m}")


def birth_death(lam: np.ndarray, mu: np.ndarray) -> BlockGenerator:
    """Scalar birth-death chain as an m=1 QBD: rate lam[i] from i to i+1,
    rate mu[i] from i to i-1 (lam[L-1] and mu[0] are ignored)."""
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    L = lam.size
    blocks = np.zeros((L, 3, 1, 1))
    blocks[:-1, 2, 0, 0] = lam[:-1]
    blocks[1:, 0, 0, 0] = mu[1:]
    sizes = np.ones(L, dtype=np.int32)
    _set_diagonal(blocks, sizes, 1)
    return BlockGenerator(L, 1, 1, blocks, sizes, f"birth_death_L{L}")


def planted_reversible(L: int, m: int, seed: int, *, b: int = 1, density: float = 0.5,
                       spread: float = 4.0, last: int | None = None):
    """Reversible chain with a planted stationary vector.

    Draw pi* > 0 and a symmetric non-negative weight matrix W supported on the
    block band; set q_ij = w_ij / pi*_i (i != j).  Then pi*_i q_ij = pi*_j q_ji
    (detailed balance), so pi* is stationary.  Returns (generator, pi*) with
    pi* normalised to sum 1.
    """
    sizes = _sizes(L, m, last)
    rng = np.random.Generator(np.random.PCG64(seed))
    N = int(sizes.sum())
    pi = np.exp(rng.uniform(-spread / 2, spread / 2, size=N))
    pi /= pi.sum()
    off = np.zeros(L + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    blocks = np.zeros((L, 2 * b + 1, m, m))
    # weights for each unordered block pair (i, i+d), d >= 0
    for i in range(L):
        for d in range(0, b + 1):
            k = i + d
            if k >= L:
                continue
            ni, nk = sizes[i], sizes[k]
            w = (rng.random((ni, nk)) < density) * rng.random((ni, nk))
            if d == 0:
                w = np.triu(w, 1)
                w = w + w.T
            elif not w.any():
                w[rng.integers(ni), rng.integers(nk)] = 1.0
            pi_i = pi[off[i]: off[i] + ni]
            pi_k = pi[off[k]: off[k] + nk]
            blocks[i, d + b, :ni, :nk] = w / pi_i[:, None]
            if d > 0:
                blocks[k, -d + b, :nk, :ni] = w.T / pi_k[:, None]
    # keep every level strongly connected inside: add a ring of small weights
    for i in range(L):
        ni = sizes[i]
        if ni < 2:
            continue
        pi_i = pi[off[i]: off[i] + ni]
        for r in range(ni):
            c = (r + 1) % ni
            wrc = 0.05
            blocks[i, b, r, c] += wrc / pi_i[r]
            blocks[i, b, c, r] += wrc / pi_i[c]
    _set_diagonal(blocks, sizes, b)
    gen = BlockGenerator(L, m, b, blocks, sizes, f"planted_L{L}_m{m}_b{b}")
    return gen, pi


def positive_start(gen: BlockGenerator, seed: int) -> np.ndarray:
    """A random strictly positive start vector (compact, length N, sums to 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.random(gen.N) + 0.1
    return x / x.sum()


def served_stream(count: int, seed: int, *, L_range=(32, 2048), m_choices=(8, 16, 32, 64),
                  rate: float = 1.0):
    """Request stream of independent QBD solves: per request (arrival time,
    L, m, seed).  Levels ~ U{L_range}, block size ~ U(m_choices), arrivals
    Poisson with the given rate (requests per second)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = rng.integers(L_range[0], L_range[1] + 1, size=count)
    ms = rng.choice(np.asarray(m_choices), size=count)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    seeds = rng.integers(1, 2**31 - 1, size=count)
    return [dict(arrival=float(t[k]), L=int(Ls[k]), m=int(ms[k]), seed=int(seeds[k]))
            for k in range(count)]
