"""CPU FP64 oracle for the CGD-EnKF analysis step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check and
the benchmark's CPU-baseline leg may import this package.  It shares no code
with the HIP library: it is a plain, slow, obviously-correct NumPy/SciPy
implementation of what the analysis computes, written from the paper:

  enkf.py     the analysis by its definitions (Section 2.3, Algorithm 1),
              Cholesky and textbook CG solves, brute-force Kalman gain,
              the reduced form (Algorithm 2) and its CG variant.
  wsnet.py    the warm-start convolutional network, FP64 forward/backward.

Every function states the passage it follows.  Notation follows the build:
n = state dimension (the paper's m), m = observation dimension (the paper's
p), N = ensemble size, S = H A the observed anomalies (the paper's Z-hat).
"""
from .enkf import *  # noqa: F401,F403
