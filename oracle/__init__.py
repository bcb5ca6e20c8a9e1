"""FP64 CPU oracle for the ridge regularization path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
executes this package; only the tests, the smoke check and the CPU baseline
leg of the benchmark may.  It shares no code with the GPU path: the only
common dependency is the seeded input generator module ``workloads``, which
holds no solver arithmetic.

Contents
--------
direct   Plain definition of the path: x(lam) = (A^T A + lam I)^-1 A^T B for
         every lam, by Cholesky factorization per lam (Section 1,
         Eq. (least-square); the closed form of Section 2.1).  This is the
         graded reference.
rng      SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a
         counter-based generator, and the draws every sketch is built from.
sketch   The four sketch families of Section 4 (Gaussian, CountSketch, SJLT,
         SRHT) built or applied densely and slowly.
ihs_bin  IHS-BIN itself in FP64, in the paper's order: interval plan
         (Section 4.2), P_S, the basis recursion of the Proposition /
         Algorithm 2 (Algorithm 5 for matrix right-hand sides), and the
         composition of Algorithm 3 / 6.  Diagnostic; the GPU basis is
         compared with it when both use the same sketch, step size and k.

Parity status: every function here is pinned by a test in tests/ against
something other than itself (a closed form, a brute-force solve, a library
routine used on a different formula, or a published test vector).
"""
