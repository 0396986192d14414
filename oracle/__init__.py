"""CPU reference oracle for the QEM E-step (test infrastructure only).

A plain, slow, FP64 numpy implementation of what the hot path computes:
massively parallel importance weighting (MPIW) over all K^n sample
combinations, its log-space contraction along plates, chains and a root
pair, the reverse pass giving per-sample marginal weights, the weighted
moments, and the EMA plus closed-form M-step of QEM.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path never calls it, and it shares no code
with the HIP library: its random-number generator, samplers, densities and
contraction are written here independently from their published definitions.

Modules
  philox    Philox4x32-10 counter-based generator and the samplers built on it.
  densities log-densities of the model and proposal families.
  mpiw      log-factors, brute-force enumeration, variable elimination,
            reverse pass, moments, EMA and M-step, and the QEM loop.
"""
from . import philox, densities, mpiw  # noqa: F401
