"""The "w/o Ortho" ablation of Online TT-ALS (oracle; test infrastructure only).

The ablation of Section 5 removes the LQ/QR orthogonalisation steps of the
sequential update and attributes the resulting error growth to ill-conditioned
Gram matrices of cores updated without normalisation.  Reading used here (the
paper names only what is removed): the right-orthogonalisation of Section
3.4.1 (normalising g and the LQ sweep) is dropped, so the right interfaces
B_k are no longer orthonormal and the exact local solution needs their Gram
matrix,

    G~_k = A_k^T X^(k) B_k^T (B_k B_k^T)^+,

while the forward sweep keeps its QR (the left interfaces A_k stay
orthonormal, and the rank rule and completions of oracle.householder apply
unchanged), R is still propagated, and g = A_{m+1}^T vec(X).  Where B_k has
fewer columns than rows (J_k < r_k; always at k = m, where B_m = g) the Gram
matrix is singular and the pseudo-inverse of a full-rank B_k is used:
(B_k B_k^T)^+ = B_k (B_k^T B_k)^{-2} B_k^T.  In exact arithmetic this projects
each slice onto the same spaces as the proposed method whenever no QR needs a
completion (the right interfaces' row spaces do not depend on their gauge);
in floating point the Gram matrices of the unnormalised right cores grow
ill-conditioned over time.  Gram systems are solved by a Cholesky
factorisation; a failed factorisation raises numpy.linalg.LinAlgError.
"""

from __future__ import annotations

import numpy as np

from .householder import householder_qr
from .ttals import (StepInfo, StreamResult, copy_state, fold, left_unfold, next_left_interface, right_interfaces,
                    right_unfold, xhat)


def _spd_solve_left(S: np.ndarray, M: np.ndarray) -> np.ndarray:
    """S^{-1} M for symmetric positive definite S (Cholesky)."""
    L = np.linalg.cholesky(S)
    return np.linalg.solve(L.T, np.linalg.solve(L, M))


def right_gram_pinv(B: np.ndarray) -> np.ndarray:
    """(B B^T)^+ for B (r x J) of full rank: (B B^T)^{-1} when r <= J, else
    B (B^T B)^{-2} B^T."""
    r, J = B.shape
    if r <= J:
        return _spd_solve_left(B @ B.T, np.eye(r))
    H = _spd_solve_left(B.T @ B, np.eye(J))
    return B @ H @ H @ B.T


def local_solve_gram(A: np.ndarray, X3: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Exact local solution with orthonormal A and general B:
    A^T X^ B^T (B B^T)^+, as r_{k-1} x I_k x r_k."""
    P, n, J = X3.shape
    T = A.T @ X3.reshape(P, n * J, order="F")              # r_{k-1} x (I_k J)
    G = T.reshape(A.shape[1] * n, J, order="F") @ B.T       # (r_{k-1} I_k) x r_k
    G = G @ right_gram_pinv(B)
    return G.reshape(A.shape[1], n, B.shape[0], order="F")


def online_step_noortho(cores, g, X, *, qr=householder_qr):
    """One update of the ablation variant.  Returns (cores, g, StepInfo)."""
    modes = [G.shape[1] for G in cores]
    m = len(cores)
    X = np.asarray(X, dtype=np.float64).reshape(modes, order="F")
    info = StepInfo(g_norm_in=float(np.linalg.norm(g)))
    cores, g = copy_state(cores, g)                 # no normalisation, no LQ sweep
    B = right_interfaces(cores, g)
    A = np.ones((1, 1))
    for k in range(1, m + 1):
        Gt = local_solve_gram(A, xhat(X, modes, k), B[k - 1])
        Q, R = qr(left_unfold(Gt))
        cores[k - 1] = fold(Q, Gt.shape)
        if k < m:
            nxt = cores[k]
            cores[k] = fold(R @ right_unfold(nxt), nxt.shape)
        else:
            g = R @ g
        A = next_left_interface(A, cores[k - 1])
    x = X.reshape(-1, order="F")
    g = A.T @ x
    M = (A @ g).reshape(modes, order="F")
    info.M = M
    info.E = float(np.linalg.norm(x - M.reshape(-1, order="F")))
    info.Xnorm = float(np.linalg.norm(x))
    info.f_final = 0.5 * info.E ** 2
    return cores, g, info


def run_stream_noortho(slices, cores0, g0, *, keep_M=False):
    """The ablation variant over a stream (see ttals.run_stream)."""
    cores, g = copy_state(cores0, g0)
    E, Xn, infos = [], [], []
    for X in slices:
        cores, g, info = online_step_noortho(cores, g, X)
        E.append(info.E)
        Xn.append(info.Xnorm)
        if not keep_M:
            info.M = None
        infos.append(info)
    return StreamResult(np.array(E), np.array(Xn), cores, g, infos)
