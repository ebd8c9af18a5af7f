"""Dense regular splittings Q^T = M - N of section 2 and their spectra.

Each M is built from its definition on the block partition of A = Q^T:
  jacobi   M = blockdiag(A_{i,i})
  gs       M = block lower triangle of A (block Gauss-Seidel)
  jgs      M = blockdiag(M_1..M_p), M_j the block lower triangle of the
           diagonal chunk of levels owned by processor j ([BB] scheme,
           Algorithm 1)
  stair1   type-1 stair matrix: odd block rows (1-based) keep A_{i,i}, even
           rows keep A_{i,i-1}, A_{i,i}, A_{i,i+1}
  stair2   type-2 stair matrix: the parities swapped
The iteration matrix is T = M^{-1} N with N = M - A.  For a singular
irreducible A the spectral radius of T is 1 and the convergence rate of the
normalised scheme is set by gamma = max{|lambda| : lambda != 1}.
"""
from __future__ import annotations

import numpy as np

from .dense import level_offsets


def splitting_M(A: np.ndarray, sizes, kind: str, chunks=None) -> np.ndarray:
    off = level_offsets(sizes)
    L = len(off) - 1
    M = np.zeros_like(A)

    def put(i, k):
        M[off[i]:off[i + 1], off[k]:off[k + 1]] = A[off[i]:off[i + 1], off[k]:off[k + 1]]

    if kind == "jacobi":
        for i in range(L):
            put(i, i)
    elif kind == "gs":
        for i in range(L):
            for k in range(i + 1):
                put(i, k)
    elif kind == "jgs":
        for start, count in chunks:
            for i in range(start, start + count):
                for k in range(start, i + 1):
                    put(i, k)
    elif kind in ("stair1", "stair2"):
        # 1-based block row r = i + 1; type 1: odd r diagonal only
        diag_only_parity = 1 if kind == "stair1" else 0
        for i in range(L):
            put(i, i)
            if (i + 1) % 2 != diag_only_parity:
                for k in (i - 1, i + 1):
                    if 0 <= k < L:
                        put(i, k)
    else:
        raise ValueError(kind)
    return M


def iteration_matrix(A: np.ndarray, sizes, kind: str, chunks=None) -> np.ndarray:
    M = splitting_M(A, sizes, kind, chunks)
    Nmat = M - A
    return np.linalg.solve(M, Nmat)


def spectrum(A: np.ndarray, sizes, kind: str, chunks=None) -> np.ndarray:
    """Eigenvalues of M^{-1} N sorted by decreasing modulus."""
    ev = np.linalg.eigvals(iteration_matrix(A, sizes, kind, chunks))
    return ev[np.argsort(-np.abs(ev), kind="stable")]


def second_modulus(ev: np.ndarray, tol: float = 1e-9) -> float:
    """gamma: largest |lambda| after removing one eigenvalue equal to 1."""
    ev = np.asarray(ev)
    j = int(np.argmin(np.abs(ev - 1.0)))
    if abs(ev[j] - 1.0) > tol:
        raise ValueError("no eigenvalue equal to 1")
    rest = np.delete(ev, j)
    return float(np.max(np.abs(rest))) if rest.size else 0.0
