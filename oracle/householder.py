"""Thin Householder QR and LQ in FP64 (oracle; test infrastructure only).

Algorithm 1 re-orthogonalises cores with a thin QR (forward sweep) and an LQ
(right-orthogonalisation); Section 3.4 notes that LQ is the QR of the
transpose.  The paper fixes no sign convention and does not discuss
rank-deficient inputs, so this oracle reads them as follows:

* diag(R) >= 0 (and so diag(L) >= 0);
* a column whose remaining part has norm <= tol * ||M||_F gets the identity
  in place of a reflector; its sub-diagonal remainder is dropped and its
  diagonal entry of R is set to 0.  The corresponding column of Q is then the
  unit vector e_j carried through the earlier reflectors, a deterministic
  orthonormal completion.  Any orthonormal completion is equally valid for the
  method's outputs.

The reflector construction is the textbook one (Householder vector
v = x + sign(x_1) ||x|| e_1, applied as I - 2 v v^T / v^T v), with Q formed by
applying the reflectors in reverse order to the first n columns of I.
"""

from __future__ import annotations

import numpy as np

EPS64 = float(np.finfo(np.float64).eps)
DEFAULT_TOL = 64.0 * EPS64


def householder_qr(M: np.ndarray, tol: float = DEFAULT_TOL):
    """Thin QR of an m x n matrix (m >= n): M = Q R, Q^T Q = I_n, diag(R) >= 0."""
    A = np.array(M, dtype=np.float64, copy=True)
    m, n = A.shape
    if m < n:
        raise ValueError("thin QR needs rows >= columns")
    thr = tol * float(np.linalg.norm(A))
    vs = []
    for j in range(n):
        x = A[j:, j]
        alpha = float(np.linalg.norm(x))
        if alpha <= thr:
            A[j:, j] = 0.0
            vs.append(None)
            continue
        v = x.copy()
        v[0] += alpha if x[0] >= 0.0 else -alpha
        vv = float(v @ v)
        # apply H = I - 2 v v^T / (v^T v) to the trailing block
        A[j:, j:] -= np.outer(v, (2.0 / vv) * (v @ A[j:, j:]))
        A[j + 1:, j] = 0.0
        vs.append((v, vv))
    R = np.triu(A[:n, :])
    Q = np.zeros((m, n))
    Q[:n, :n] = np.eye(n)
    for j in range(n - 1, -1, -1):
        if vs[j] is None:
            continue
        v, vv = vs[j]
        Q[j:, :] -= np.outer(v, (2.0 / vv) * (v @ Q[j:, :]))
    s = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


def lq(M: np.ndarray, tol: float = DEFAULT_TOL):
    """LQ of an m x n matrix (m <= n) as the QR of its transpose: M = L Q,
    L lower triangular with diag(L) >= 0, Q Q^T = I_m.  Returns (L, Q)."""
    Qt, Rt = householder_qr(np.asarray(M).T, tol)
    return Rt.T, Qt.T
