"""Plain, slow FP64 CPU oracle for the block staircase-splitting solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
anything in this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP library.

Contents (each function cites the passage it follows):
  dense.py            the problem statement (eq. (1)): assembling Q^T, the
                      residual ||Q^T x||_1, the reference solution by a dense
                      null-space solve for tiny chains.
  gth.py              Grassmann-Taksar-Heyman elimination (textbook; the
                      paper does not use it) - the reference pi for N <~ 4096.
  level_reduction.py  block (level-by-level) GTH for block-banded Q - the
                      reference pi for large chains.
  staircase.py        Algorithm 2 (STAIR1 / STAIR2) and Algorithm 1 (JGS)
                      written from section 2, in FP64 with LU block solves,
                      on block-banded generators (BlockSystem) and on
                      generators of any block pattern (SparseBlockSystem).
  splittings.py       the dense regular splittings Q^T = M - N of section 2
                      (block Jacobi, block Gauss-Seidel, the [BB] composite,
                      stair matrices M1 / M2) and their iteration spectra.
  csweep.c            the same Algorithm 2 sweep as plain C with OpenMP loops
                      over levels (mirrors the paper's C++/OpenMP build): the
                      CPU baseline, and the whole-chain reference of the
                      full-size parity tests.
  krylov.py           restarted GMRES on (I - M^{-1} N) x = 0, the splitting
                      as a preconditioner (the paper's stated future work).
  table1.py           Example 3 / Table 1: the spectral gaps (gamma, the
                      largest modulus after 1) of the block Jacobi, block
                      Gauss-Seidel and staircase iterations, and the ratios
                      rho_1, rho_2 over random trials.

Every function here is pinned by tests under tests/ against facts that do not
come from the oracle itself (closed forms, the paper's worked examples,
brute-force solves, planted solutions, spectral identities).
"""
