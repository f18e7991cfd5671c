"""CPU oracle for finite-precision (block-Jacobi preconditioned) CG detection.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU path.

Contents
  rounding  -- fl(.) operator (Def. 1-2, Table I): round-to-nearest-even into
               fp32 / bf16 / fp16 / fp8-e4m3fn with gradual underflow.
  detect    -- the plain definition (eq. inversion: A = H^H H + sigma^2 I,
               b = H^H y, x = A^{-1} b by Cholesky), Alg. 1 (CG), Alg. 2
               (FP-CG), eq. pre_BJ and Alg. 3 (FP-BJ-CG) step by step, the
               emulated precision schedule, FP64 residual refresh, FP64
               iterative refinement, the QAM slicer and bit-error counting.
  demap     -- soft output after detection: the effective gain of each
               user from eq. pre_BJ's block inverses and max-log LLRs over the
               Gray QAM points (readings in its header), with the exact LLRs
               of the same model for the pins.
  theory    -- unit roundoffs, gamma_n (eq. gamma), the attainable-accuracy
               bounds of Thm 2 / Thm 4, the precision heuristic (eq. heuristic,
               eq. heuristic_bj), the Gram-entry moments of App. B and the
               multiplication-count cost model of Sec. V.

Every function is pinned by a CPU test in tests/ against something other than
itself (exact arithmetic, closed forms, library routines, the paper's printed
numbers).  Functions without such a pin say "parity unpinned".
"""
