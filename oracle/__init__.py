"""FP64 CPU oracle for batched emulator posterior sampling (test infrastructure only).

This package is the plain, slow, obviously-correct reference that the HIP path is checked
against.  It is NOT part of the product: only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import it.  It shares no code with the HIP library and
imports nothing from it; the only common code is the seeded input generator `workloads`,
which holds no sampler arithmetic.

Everything is numpy in float64, vectorised over chains, following the paper's definitions:

  philox   counter-based generator (Salmon et al., SC'11) and its uniform/normal maps
  mlp      the tanh MLP emulator, its input gradient (reverse mode) and weight gradients
  target   log-density: Gaussian (+ twist) + coef*MLP, box prior, plain spectrum model,
           and the whitened density of Sec. 2.2 (Alg. 1 / eq. log_prob_transform)
  samplers MH, MALA (Sec. 2.1), HMC leapfrog (eq. hamiltonian), AIES stretch move (Sec. 2.3)
  adapt    ensemble covariance, jittered Cholesky (Sec. 3.2), dual-averaging step size
  ess      multi-chain effective sample size (Geyer initial monotone sequence)
  train    MSE + Adam training of the emulator, importance weights, Kish ESS

Functions whose result no test pins independently say "parity unpinned" in their docstring.
"""
