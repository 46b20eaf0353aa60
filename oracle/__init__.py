"""CPU oracle for the FDE-constrained ADMM method -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy/SciPy implementation of what the GPU path computes,
written from the paper (Pougkakiotis, Pearson, Leveque, Gondzio, "Fast
Solution Methods for Convex Fractional Differential Equation Optimization").
It applies every structured matrix as a dense 1-D factor (no FFT anywhere):
Toeplitz products are dense matrix products along lines, the circulant
preconditioner is applied with explicit DFT matrices.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never calls it and shares
no code with it; the only shared module is ``workloads`` (seeded inputs).

Modules
    grunwald  -- fractional binomial weights and their derivatives (Sec. 4)
    operator  -- the constraint matrix D of eq. (4.9), line-wise and dense
    precond   -- T. Chan circulants and the Schur-complement preconditioner
                 (Sec. 5, eq. (5.2); Sec. 3.2, eq. (3.10))
    admm      -- Algorithm 1 with the merged x-step / normal equations (Sec. 3.1)
    kkt       -- objective, KKT residuals, dual infeasibility, active-set polish
    grad      -- gradients of the optimal value (envelope theorem on eq. (3.5))

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against closed forms, dense brute force, invariants or a library routine,
except the FP32-preconditioner error figure, which is a reported quantity
("parity unpinned" beyond the stated bound).
"""
