"""FP64 CPU oracle for randomized block BFGS matrix inversion.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this package; only
the tests, the smoke check and the benchmark's CPU-baseline leg use it.  It shares
no code with the GPU implementation: the only thing both sides agree on is the
published definition of the counter-based sketch stream (Philox4x64-10, Box-Muller,
Floyd sampling), which each side implements on its own.

Modules
  philox   Philox4x64-10 block function (Salmon et al., SC'11).
  sketch   Gaussian and coordinate sketches drawn from that stream.
  rbfgs    fixed-sketch RBFGS (eq. qunac, Sec. 8.7) and AdaRBFGS (Alg. 4 /
           eq. Cholimprov, Sec. 9.3), residuals and the per-step estimator.
  variants simultaneous randomized Kaczmarz (eq. badbroyadj), AIP (eq. BFGSas)
           and randomized PSB (eq. Xupdatesym with W = I), and the residual
           estimator of the row variants.
  comparison  Newton-Schulz (eq. Newton-Schulz) and MR (eq. MRiter) with the starting
           points of Sec. 10, and the power-method norm estimate they use.
  ridge    the ridge-regression Hessian scale B^T B + lam I (eq. ridgeMatrix).
  pcg      preconditioned CG for A x = b with X ~ A^-1 as the preconditioner.
  partition  partition sampling with the probabilities of eq. (ihsih0) for fixed
           RBFGS and AdaRBFGS (Sec. 9.3), the draw from the stream, the
           Horvitz-Thompson residual estimator, and Kaczmarz with the importance
           probabilities of eq. (discoptprob) taking X_k as the proxy for A^-1.
  theory   closed-form quantities used by the pins: the rate rho of Thm 6.2 /
           eq. rhoequiv, E[Z] for discrete sketches (Prop. 7.1), brute-force
           projections (eq. NF, eq. NFsym) by a dense KKT solve.

Parity status: every function here is pinned by a `-m "not gpu"` test against
something other than itself (see tests/test_oracle_pins.py, tests/test_oracle_variants.py,
tests/test_oracle_comparison.py, tests/test_oracle_ridge.py,
tests/test_oracle_pcg.py, tests/test_oracle_partition.py).
"""
