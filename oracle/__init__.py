"""FP64 CPU oracle for the Monte Carlo Shiftable Filter (MCSF).

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke entry
point and the benchmark's CPU-baseline leg may import it.  The product path
(the HIP library and its Python binding) never imports, links or calls
anything here, and this package imports nothing from the product path.

Contents
--------
philox : the Philox4x32-10 counter-based generator, written from its published
         definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
         easy as 1, 2, 3", SC'11).
mcsf   : whitening, order rule, term sampling, and the four reference filters
         (direct exact filter, direct filter with the sampled kernel, the
         separable MCSF of Algorithm 1, and the full unsampled expansion).

Every function cites the passage of the paper (Ghosh & Chaudhury, "Fast
Bilateral Filtering of Vector-Valued Images", arXiv 1605.02164) it follows.
Pins for each function live in ``tests/test_oracle_*.py``.
"""

from . import philox, mcsf  # noqa: F401
