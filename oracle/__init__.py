"""FP64 CPU oracle for the Online TT-ALS per-slice update.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product path
(the HIP library and its Python binding) never imports, calls or links it, and
this package never imports the product path.

Contents
  householder  thin Householder QR / LQ with the rank-deficiency rule
  ttals        Algorithm 1 (Online TT-ALS) taken literally, with instrumentation
  ttsvd        batch TT-SVD, used only as a brute-force comparison
  metrics      reconstruction error of a stream (Section 5.1)
  closed_form  the order-3 closed form of the method's outputs (a derived pin)

Parity status: every function is pinned by tests under tests/ against
properties the paper and the mathematics fix (orthogonality, gauge invariance,
least-squares stationarity, Proposition 1's identity, exact recovery,
Eckart-Young bounds, an order-3 closed form).  Raw core entries are not
pinned: they are unique only up to an orthogonal gauge per bond.
"""

from . import householder, ttals, ttsvd, metrics, closed_form  # noqa: F401
