"""CPU FP64 oracle for SLSE-FRS (Chen, Xie, Yang, "Sequential Least-Squares
Estimators with Fast Randomized Sketching for Linear Statistical Models").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU library computes.  Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the HIP library (no kernels, headers, constants or
helpers); both sides implement the counter-based generator (Philox4x64-10) and
the keyed permutation from their published definitions.

Modules
  rng     Philox4x64-10, the stream map, Rademacher signs, a Feistel PRP with
          cycle walking, CountSketch hashes and Box-Muller Gaussians.
  fwht    Sylvester-order unnormalised Walsh-Hadamard transform.
  sketch  SRHT / CountSketch / Gaussian sketches of the tall data [X|Y]
          (Sec. 3, the efficient construction and Alg. 2).
  ols     Householder-QR OLS (the closed form of the problem statement) and a
          corrected-seminormal refinement in extended precision.
  slse    The SLSE-FRS iteration of Alg. 2 with M-IHS steps, eqs. (98)/(99).
  adjoint Adjoint of the OLS map beta_hat(X, Y) for L = w^T beta_hat.

Every function states the passage of the paper it follows.  Functions without
a pin say "parity unpinned" in their docstring (none at present).
"""
