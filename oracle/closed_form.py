"""Order-3 closed form of the method's output (oracle; test infrastructure only).

For a stream of matrices X_t (I_1 x I_2, i.e. n = 3) the update's output slice
depends only on a subspace recursion.  Derivation (from Algorithm 1 and Eq. 5):
after the forward sweep M_t = U_t U_t^T X_t with U_t = G_1[t] (the first core is
the left interface of the last one, and the final least-squares step projects
onto it); G_1[t] spans the range of X_t B_1^T, and B_1 at time t equals, up to an
invertible r_1 x r_1 factor from the LQ sweep, U_{t-1}^T X_{t-1}.  Hence

    U_1 = orth(X_1 B_0^T),  B_0 = G_2[0] x_3 g[0]   (initial cores),
    U_t = orth(X_t X_{t-1}^T U_{t-1}),               t >= 2,
    M_t = U_t U_t^T X_t.

This is one step of a cross-Gram subspace iteration per slice.  It is computed
here with numpy's SVD as the orthonormal-basis routine, independently of the
Householder QR, LQ, interfaces and sweeps of the literal oracle.
"""

from __future__ import annotations

import numpy as np


def _orth(M: np.ndarray) -> np.ndarray:
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    return U


def order3_outputs(slices, G2_init: np.ndarray, g_init: np.ndarray):
    """Yield M_t for a stream of I_1 x I_2 slices and initial cores (G_2, g)."""
    r1, I2, r2 = G2_init.shape
    B0 = (G2_init.reshape(r1 * I2, r2, order="F") @ g_init).reshape(r1, I2, order="F")
    U = None
    prev = None
    for X in slices:
        X = np.asarray(X, dtype=np.float64)
        if U is None:
            U = _orth(X @ B0.T)
        else:
            U = _orth(X @ (prev.T @ U))
        yield U @ (U.T @ X)
        prev = X
