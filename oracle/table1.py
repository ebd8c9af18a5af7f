"""Example 3 / Table 1 of section 2, on the CPU: spectral gaps of block
Jacobi (BJ), block Gauss-Seidel (BGS) and block staircase (BS, type 1)
splittings of random singular M-matrices in banded block lower Hessenberg
form.

TEST INFRASTRUCTURE: an experiment on the oracle's dense splittings
(splittings.py, pinned by tests/test_oracle_pins.py); nothing in the product
path uses it.

For every trial and partition size kp the iteration matrices M^{-1} N of the
three splittings are formed densely and gamma (the largest modulus after the
eigenvalue 1) is taken from their full spectra.  The table reports, over the
trials, the largest rho_1 = log(1/gamma_BGS) / log(1/gamma_BJ) and
rho_2 = log(1/gamma_BGS) / log(1/gamma_BS), with rho_1 = inf when block Jacobi
has a second eigenvalue of modulus 1 (it does not converge).

Readings (the printed table is partly empty and its caption says k = 64,
n = 16 while its columns run over k = 16, 32, 64): the matrix has n = 16
blocks of size k, so N = 16 k; the partitions kp in {16, 32, 64} are those of
the printed rows; the cells computed are the printed ones (kp = 16 and 32 at
k = 64, kp = 64 at every k).

    python -m oracle.table1 --trials 1000 --workers 8
"""
from __future__ import annotations

import argparse
import math
import time

import numpy as np

from . import splittings

CELLS = [(16, 64), (32, 64), (64, 16), (64, 32), (64, 64)]   # (kp, k)
KINDS = ("jacobi", "gs", "stair1")


def gammas(A: np.ndarray, sizes) -> dict:
    """gamma of each splitting kind for the block partition `sizes`."""
    return {kind: splittings.second_modulus(splittings.spectrum(A, sizes, kind))
            for kind in KINDS}


def ratios(g: dict) -> tuple[float, float]:
    """(rho_1, rho_2) from the gammas of one matrix and partition."""
    gs = math.log(1.0 / g["gs"])
    bj = g["jacobi"]
    rho1 = math.inf if bj >= 1.0 - 1e-10 else gs / math.log(1.0 / bj)
    rho2 = gs / math.log(1.0 / g["stair1"])
    return rho1, rho2


def _trial(args):
    seed, cells = args
    from threadpoolctl import threadpool_limits

    import synth
    out = []
    with threadpool_limits(1):
        for kp, k in cells:
            g = synth.hessenberg_mmatrix(16, k, seed)
            A = g.to_scipy().T.toarray()
            sizes = synth.equal_levels(g.N, kp)
            gm = gammas(A, sizes)
            out.append((kp, k, gm, ratios(gm)))
    return seed, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trials", type=int, default=20)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--seed0", type=int, default=0)
    args = ap.parse_args()
    from multiprocessing import get_context
    t0 = time.perf_counter()
    best = {c: [0.0, 0.0] for c in CELLS}
    gam = {c: {kind: [] for kind in KINDS} for c in CELLS}
    jobs = [(args.seed0 + t, CELLS) for t in range(args.trials)]
    with get_context("fork").Pool(args.workers) as pool:
        for _seed, out in pool.imap_unordered(_trial, jobs):
            for kp, k, gm, (r1, r2) in out:
                c = (kp, k)
                best[c][0] = max(best[c][0], r1)
                best[c][1] = max(best[c][1], r2)
                for kind in KINDS:
                    gam[c][kind].append(gm[kind])
    dt = time.perf_counter() - t0
    print(f"Example 3 / Table 1: {args.trials} trials (seeds {args.seed0}.."
          f"{args.seed0 + args.trials - 1}), n = 16 blocks of size k, lower bandwidth 4k; "
          f"{dt:.0f} s on {args.workers} workers\n")
    print("| kp | k | max rho_1 | max rho_2 | median gamma BJ | median gamma BGS | median gamma BS |")
    print("|---|---|---|---|---|---|---|")
    for c in CELLS:
        kp, k = c
        r1 = "inf" if math.isinf(best[c][0]) else f"{best[c][0]:.2f}"
        med = {kind: float(np.median(gam[c][kind])) for kind in KINDS}
        print(f"| {kp} | {k} | {r1} | {best[c][1]:.2f} | {med['jacobi']:.4f} | {med['gs']:.4f} | "
              f"{med['stair1']:.4f} |")


if __name__ == "__main__":
    main()
