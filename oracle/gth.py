"""Dense Grassmann-Taksar-Heyman (GTH) elimination.

Textbook state reduction for the stationary vector of an irreducible CTMC
(the paper cites surveys of such direct methods in section 1 but does not use
GTH).  It reads only off-diagonal rates and never subtracts, so every
quantity is formed from non-negative terms.

Eliminating the last remaining state k gives the censored chain on states
0..k-1 with rates q_ij + q_ik q_kj / s_k, where s_k = sum_{j<k} q_kj is the
rate out of k into the remaining states.  Back substitution then gives
pi_k = sum_{i<k} pi_i q_ik / s_k starting from pi_0 = 1.
"""
from __future__ import annotations

import numpy as np


def gth(Q: np.ndarray) -> np.ndarray:
    """Stationary vector of the generator Q (rows of Q sum to 0), FP64."""
    A = np.array(Q, dtype=np.float64, copy=True)
    N = A.shape[0]
    for k in range(N - 1, 0, -1):
        s = A[k, :k].sum()
        if not s > 0.0:
            raise ValueError(f"GTH: state {k} has no rate into states < {k}; "
                             "the generator is reducible")
        A[:k, k] /= s
        A[:k, :k] += np.outer(A[:k, k], A[k, :k])
    pi = np.zeros(N)
    pi[0] = 1.0
    for k in range(1, N):
        pi[k] = pi[:k] @ A[:k, k]
    return pi / pi.sum()
