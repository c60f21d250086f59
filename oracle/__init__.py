"""Plain FP64 CPU oracle for one MPPI iteration with covariance-variable importance
sampling (Williams, Aldrich & Theodorou, arXiv 1509.01149).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP library and
its Python binding) never imports, links or executes anything in here, and this
package imports nothing from the product path.  The two sides share only the seeded
input generators in ``workloads``.

Everything is written for readability against the paper, not speed: FP64 NumPy,
vectorised over the K samples, a Python loop over time.  Each function names the
section / equation / algorithm of the paper it follows.
"""
from . import philox, noise, systems, mppi, lqr, mlp  # noqa: F401
