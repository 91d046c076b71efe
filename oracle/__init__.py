"""FP64 CPU oracle of the two-range pseudopotential LBM step (arXiv:1806.06943).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package, and this package never imports the product.
"""
from .oracle import *  # noqa: F401,F403
