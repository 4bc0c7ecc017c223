"""FP64 CPU oracle for the Seed-CG hot path -- TEST INFRASTRUCTURE, not the product.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import,
call, link or run anything in this package.  It shares no code with the HIP
library: its Wilson operator is a plain C loop (wilson_ref.c) and its solvers
(seedcg.py) follow the paper's Algorithm 1 and textbook CG step by step in NumPy.

Parity status of each part (what pins it is listed in the tests):
  * gamma matrices, Wilson D, A, A^dag, M ........ pinned (Clifford algebra, free-field
    closed-form spectra, gamma5-hermiticity, gauge covariance, a second dense build)
  * Algorithm 1 (Seed-CG with periodic reorth) ... pinned (T = LU of Eq. 2, T from CG
    coefficients, D-Lanczos iterate = CG iterate, Galerkin identity of Eq. 1,
    k = 1 exact Galerkin, linearity, duplicate right-hand sides)
  * plain CG ..................................... pinned (dense Cholesky solve)
"""
