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

Safeguard (not from the paper).  When the chain drifts strongly across its
levels, T is far from normal: over a short cycle the 2-norm that GMRES
minimises can stall, or ||Q^T x||_1 can even grow, while the plain iteration
still makes progress.  A cycle is therefore kept only if it lowers
||Q^T x||_1 clearly faster than plain steps: per application of T, by at
least the square of the factor the last block of plain steps achieved
(before any plain block has run: by half over the cycle).  Otherwise the
iterate stays and k plain applications of T follow (normalised every 16 and
at the end), with k = restart at first and doubled after every rejected
cycle; their factor becomes the new yardstick.
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


NORM_EVERY = 16     # plain applications between normalisations


def plain_steps(sys, x: np.ndarray, k: int, stair_type: int = 1) -> np.ndarray:
    """k applications of T, normalised every NORM_EVERY and at the end."""
    for t in range(k):
        x = stair_apply(sys, x, stair_type)
        if (t + 1) % NORM_EVERY == 0:
            x = x / x.sum()
    return x / x.sum()


def gmres_solve(sys, *, restart: int = 30, tol: float = 1e-12, maxit: int = 10_000,
                stair_type: int = 1, x0: np.ndarray | None = None) -> KrylovResult:
    """Safeguarded restarted GMRES on (I - M^{-1} N) x = 0 until
    ||Q^T x||_1 <= tol or maxit applications of T."""
    x = np.full(sys.N, 1.0 / sys.N) if x0 is None else np.asarray(x0, float) / np.sum(x0)
    applies, cycles, hist = 0, 0, []
    res = sys.residual(x)
    k = restart
    plain_rate = None   # residual factor per application of the last plain block
    while res > tol and applies + 2 <= maxit:
        xn, a, _ = gmres_cycle(sys, x, min(restart, maxit - applies - 1), stair_type)
        applies += a
        cycles += 1
        rn = sys.residual(xn)
        need = 0.5 ** (1.0 / a) if plain_rate is None else plain_rate ** 2
        if rn < res and (rn / res) ** (1.0 / a) <= need:
            x, res = xn, rn
        else:
            steps = min(k, maxit - applies)
            if steps > 0:
                x = plain_steps(sys, x, steps, stair_type)
                applies += steps
                rp = sys.residual(x)
                plain_rate = (rp / res) ** (1.0 / steps) if res > 0.0 else 1.0
                res = rp
            k *= 2
        hist.append(res)
    return KrylovResult(x, applies, cycles, res, res <= tol, hist)
