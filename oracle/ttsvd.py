"""Batch TT-SVD (oracle; test infrastructure only).

The paper cites TT-SVD (Section 1.1) as the basic batch method: sequential
truncated SVDs of the unfoldings of the whole tensor.  It is written here from
that definition and used only as a brute-force comparison for the online
method on small streams.
"""

from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def tt_svd(X: np.ndarray, ranks: Sequence[int]) -> Tuple[List[np.ndarray], List[float]]:
    """TT decomposition of an order-d tensor with TT-ranks (r_1..r_{d-1}).

    Returns the cores (r_{k-1}, I_k, r_k) and the Frobenius norms of the
    singular values discarded at each of the d-1 truncations.  The error is
    bounded by sqrt(sum of their squares)."""
    X = np.asarray(X, dtype=np.float64)
    dims = X.shape
    d = len(dims)
    assert len(ranks) == d - 1
    cores, tails = [], []
    C = X.reshape(-1, order="F")
    r_prev = 1
    for k in range(d - 1):
        C = C.reshape(r_prev * dims[k], -1, order="F")
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        rk = min(int(ranks[k]), s.size)
        tails.append(float(np.sqrt(np.sum(s[rk:] ** 2))))
        cores.append(U[:, :rk].reshape(r_prev, dims[k], rk, order="F"))
        C = s[:rk, None] * Vt[:rk, :]
        r_prev = rk
    cores.append(C.reshape(r_prev, dims[-1], 1, order="F"))
    return cores, tails


def tt_to_full(cores: Sequence[np.ndarray]) -> np.ndarray:
    acc = np.ones((1, 1))
    for c in cores:
        r0, n, r1 = c.shape
        acc = (acc @ c.reshape(r0, n * r1, order="F")).reshape(-1, r1, order="F")
    return acc[:, 0].reshape([c.shape[1] for c in cores], order="F")


def unfolding_tail(X: np.ndarray, k: int, r: int) -> float:
    """Eckart-Young: norm of the singular values beyond r of the unfolding
    (I_1..I_k) x (I_{k+1}..I_d); the best rank-r error of that unfolding."""
    X = np.asarray(X, dtype=np.float64)
    P = int(np.prod(X.shape[:k]))
    s = np.linalg.svd(X.reshape(P, -1, order="F"), compute_uv=False)
    return float(np.sqrt(np.sum(s[r:] ** 2)))
