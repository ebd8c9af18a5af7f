"""Krylov acceleration of the block staircase splitting, FP64.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports or runs it.

The Conclusions name the use of staircase splittings as preconditioners as
future work, and the Introduction recalls splittings preconditioning
projection methods such as GMRES.  This is that combination written from
the textbook definitions: restarted GMRES (Saad and Schultz) on the
left-preconditioned singular system

    B x = 0,   B = M^{-1} A = I - T,   T = M^{-1} N,

for the stair splitting A = Q^T = M - N of section 2 (T is applied by the
three parallel loops of Algorithm 2 without normalisation, stair_apply).
Each cycle starts from the normalised iterate x (e^T x = 1):
  r = -B x = T x - x,  beta = ||r||_2,  v_1 = r / beta;
  Arnoldi (modified Gram-Schmidt) gives V_{j+1} and the (j+1) x j Hessenberg
  H_j with B V_j = V_{j+1} H_j;
  y minimises ||beta e_1 - H_j y||_2 (a library least-squares solve);
  x <- x + V_j y, then x <- x / e^T x.
Cycles repeat until ||Q^T x||_1 <= tol or maxit applications of T.  Since 1 is
a simple eigenvalue of T, GMRES drives B x to 0 along the null vector pi.
Every cycle is kept: this is plain restarted GMRES, with no rule of its own
for rejecting a cycle.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .staircase import stair_apply


@dataclass
class KrylovResult:
    x: np.ndarray
    applies: int          # applications of T
    cycles: int
    residual: float       # ||Q^T x||_1 of the normalised x
    converged: bool
    history: list = field(default_factory=list)   # residual after each cycle


def gmres_cycle(sys, x: np.ndarray, restart: int, stair_type: int = 1):
    """One GMRES(restart) cycle from x; returns (x_new normalised, applies,
    the least-squares residual estimates ||beta e1 - H_j y_j||_2 per step)."""
    n = x.size
    r = stair_apply(sys, x, stair_type) - x
    beta = float(np.linalg.norm(r))
    if beta == 0.0:
        return x / x.sum(), 1, [0.0]
    V = np.zeros((restart + 1, n))
    H = np.zeros((restart + 1, restart))
    V[0] = r / beta
    applies = 1
    est = []
    j_used = 0
    for j in range(restart):
        w = V[j] - stair_apply(sys, V[j], stair_type)     # B v_j
        applies += 1
        for i in range(j + 1):
            H[i, j] = float(V[i] @ w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = float(np.linalg.norm(w))
        j_used = j + 1
        e1 = np.zeros(j + 2)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)
        est.append(float(np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y)))
        if H[j + 1, j] <= 1e-300:
            break
        V[j + 1] = w / H[j + 1, j]
    e1 = np.zeros(j_used + 1)
    e1[0] = beta
    y, *_ = np.linalg.lstsq(H[: j_used + 1, :j_used], e1, rcond=None)
    x_new = x + V[:j_used].T @ y
    return x_new / x_new.sum(), applies, est


def gmres_solve(sys, *, restart: int = 30, tol: float = 1e-12, maxit: int = 10_000,
                stair_type: int = 1, x0: np.ndarray | None = None) -> KrylovResult:
    """Restarted GMRES on (I - M^{-1} N) x = 0: cycles from the normalised
    iterate until ||Q^T x||_1 <= tol or maxit applications of T (a cycle that
    would exceed the budget is shortened to fit it)."""
    x = np.full(sys.N, 1.0 / sys.N) if x0 is None else np.asarray(x0, float) / np.sum(x0)
    applies, cycles, hist = 0, 0, []
    res = sys.residual(x)
    while res > tol and applies + 2 <= maxit:
        x, a, _ = gmres_cycle(sys, x, min(restart, maxit - applies - 1), stair_type)
        applies += a
        cycles += 1
        res = sys.residual(x)
        hist.append(res)
    return KrylovResult(x, applies, cycles, res, res <= tol, hist)
