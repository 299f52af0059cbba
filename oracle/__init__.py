"""FP64 CPU oracle for the block Vecchia log-likelihood.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call,
link or execute anything in this package: only the test-suite, the smoke
check and the benchmark's CPU-baseline leg use it.  It shares no code with
the HIP library (no headers, kernels, helpers or tables); the only common
dependency is the seeded input generator module ``workloads``.

Contents (each function cites the passage of the paper it follows):
  matern      - Matern covariance, eq. (maternkernel), plus the additive nugget;
                d rho / d nu from the integral form of K_nu
  preprocess  - K-means (Section 2.1), random block order, block nearest
                neighbours of each block centroid among earlier blocks
  loglik      - block terms of eq. (vecchia-vector) by their definition (joint
                minus neighbour Gaussian log-density); exact GP, eq. (likeli);
                classic Vecchia;
                trace-formula gradient (also in nu); KL divergence, eq.
                (kl-gaussian-vecchia)
  coracle     - the same block terms and gradient in plain C with OpenMP over
                blocks (csrc/bv_oracle.c), for the larger workloads
  simulate    - exact-GP and sequential-Vecchia data simulators
  ordering    - Morton, Hilbert, KD-tree and maxmin block orderings (Section 2.1)
  learned     - binned empirical variogram and an FP64 MLP forward/backward
  predict     - block Vecchia prediction (Alg. 2) and univariate conditional
                simulation with PICP / MSPE
"""
