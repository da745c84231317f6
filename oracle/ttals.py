"""Online TT-ALS, Algorithm 1, taken literally in FP64 (oracle; test only).

Notation (Sections 2-3): a stream of slices X_t of shape (I_1, ..., I_m),
m = n - 1 slice modes; cores G_k of shape (r_{k-1}, I_k, r_k), r_0 = 1; the
temporal core's newest column g (r_m entries).  Matricisation is column-major
(first index fastest, Section 2.1):
  left unfolding  of G_k: (r_{k-1} I_k) x r_k
  right unfolding of G_k: r_{k-1} x (I_k r_k)
  A_k: (I_1..I_{k-1}) x r_{k-1}, the contraction of G_1..G_{k-1} (A_1 = 1)
  B_k: r_k x (I_{k+1}..I_m), the contraction of G_{k+1}..G_m and g (B_m = g)

One update (Algorithm 1's loop body, Section 3.4):
  1. normalise g and absorb its norm into G_m; LQ sweep k = m..2, each
     G_k <- Fold(Q), G_{k-1} <- G_{k-1} x_3 L          (right-orthogonalisation)
  2. B_m = g, B_k = G_{k+1} x_3 B_{k+1}                (right interfaces)
  3. for k = 1..m: G~_k = A_k^T x X x B_k^T (Eq. 5), QR of its left unfolding,
     G_k <- Fold(Q), R propagated into G_{k+1} (or g at k = m),
     A_{k+1} = A_k x G_k                                (forward sweep)
  4. g <- A_{m+1}^T vec(X)                              (temporal row)

Every contraction is formed literally: A_k and B_k as explicit matrices, the
local solve as (A_k^T X) then times B_k^T.  No reassociation.

Readings where the paper is silent (listed with their reasons in the design
notes): the trailing mode of X_t and B_k has size 1 (one slice per step); an
all-zero g is replaced by e_1 and nothing is absorbed; QR/LQ signs and the
rank-deficient completion follow oracle.householder.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

from .householder import householder_qr, lq as _lq


# ---------------------------------------------------------------- reshapes
def left_unfold(G: np.ndarray) -> np.ndarray:
    r0, n, r1 = G.shape
    return G.reshape(r0 * n, r1, order="F")


def right_unfold(G: np.ndarray) -> np.ndarray:
    r0, n, r1 = G.shape
    return G.reshape(r0, n * r1, order="F")


def fold(M: np.ndarray, shape) -> np.ndarray:
    return np.asarray(M).reshape(shape, order="F")


# ---------------------------------------------------------------- ranks
def clamp_ranks(modes: Sequence[int], ranks: Sequence[int]) -> List[int]:
    """Largest ranks <= the requested ones for which every core update is a
    thin QR and every right-orthogonalisation step a thin LQ:
    r_k <= r_{k-1} I_k (QR of the left unfolding) and r_{k-1} <= I_k r_k (LQ of
    the right unfolding), r_0 = 1.  The paper does not discuss feasibility."""
    m = len(modes)
    r = [1] + [int(v) for v in ranks]
    for k in range(1, m + 1):
        r[k] = min(r[k], r[k - 1] * int(modes[k - 1]))
    for k in range(m, 1, -1):
        r[k - 1] = min(r[k - 1], int(modes[k - 1]) * r[k])
    return r[1:]


def check_ranks(modes: Sequence[int], ranks: Sequence[int]) -> None:
    if len(modes) < 1 or len(ranks) != len(modes):
        raise ValueError("need m >= 1 slice modes and m ranks")
    if any(int(v) < 1 for v in modes) or any(int(v) < 1 for v in ranks):
        raise ValueError("mode sizes and ranks must be >= 1")
    if list(clamp_ranks(modes, ranks)) != [int(v) for v in ranks]:
        raise ValueError("infeasible TT-ranks for these mode sizes")


# ---------------------------------------------------------------- state
@dataclass
class StepInfo:
    """Diagnostics of one update (all FP64)."""
    f_before: List[float] = field(default_factory=list)   # f(G_k) before the local solve
    f_after: List[float] = field(default_factory=list)    # f(G~_k)
    f_final: float = float("nan")                          # 1/2 ||X - M_t||^2
    g_norm_in: float = float("nan")                        # ||g|| entering the step
    M: Optional[np.ndarray] = None                         # reconstruction M_t
    E: float = float("nan")                                # ||X - M_t||_F
    Xnorm: float = float("nan")                            # ||X||_F
    B: Optional[List[np.ndarray]] = None                   # right interfaces used
    A: Optional[List[np.ndarray]] = None                   # left interfaces built
    Gtilde: Optional[List[np.ndarray]] = None              # local solutions (Eq. 5)
    right_cores: Optional[List[np.ndarray]] = None         # cores after right-orth.


def copy_state(cores, g):
    return [np.array(c, dtype=np.float64, copy=True) for c in cores], np.array(g, dtype=np.float64, copy=True)


def normalize_g(cores, g):
    """Normalise g and absorb its norm into G_m (Section 3.4.1).  An all-zero g
    (e.g. after an all-zero slice) is replaced by e_1 with nothing absorbed."""
    nu = float(np.linalg.norm(g))
    if nu > 0.0:
        cores[-1] = cores[-1] * nu
        g = g / nu
    else:
        g = np.zeros_like(g)
        g[0] = 1.0
    return cores, g, nu


def right_orthogonalize(cores, g, lq=_lq):
    """Right-orthogonalisation (Section 3.4.1): after it, G_2..G_m are
    right-orthogonal and ||g|| = 1, and the represented tensor is unchanged."""
    cores, g = copy_state(cores, g)
    cores, g, nu = normalize_g(cores, g)
    for k in range(len(cores) - 1, 0, -1):          # cores[k] is G_{k+1}
        L, Q = lq(right_unfold(cores[k]))
        cores[k] = fold(Q, cores[k].shape)
        prev = cores[k - 1]
        cores[k - 1] = fold(left_unfold(prev) @ L, prev.shape)
    return cores, g, nu


def right_interfaces(cores, g) -> List[np.ndarray]:
    """B_m = g; B_k = G_{k+1} x_3 B_{k+1} for k = m-1..1 (returned B[0..m-1]
    with B[k-1] = B_k of shape r_k x (I_{k+1}..I_m))."""
    m = len(cores)
    B: List[np.ndarray] = [None] * m
    B[m - 1] = np.asarray(g, dtype=np.float64).reshape(-1, 1)
    for k in range(m - 1, 0, -1):                   # build B_k from G_{k+1}, B_{k+1}
        G = cores[k]
        r0, n, _ = G.shape
        prod = left_unfold(G) @ B[k]                # (r_k I_{k+1}) x J_{k+1}
        B[k - 1] = prod.reshape(r0, n * B[k].shape[1], order="F")
    return B


def next_left_interface(A: np.ndarray, G: np.ndarray) -> np.ndarray:
    """A_{k+1} = A_k x_k G_k: rows (i_1..i_k) first index fastest, cols r_k."""
    r0, n, r1 = G.shape
    return (A @ right_unfold(G)).reshape(A.shape[0] * n, r1, order="F")


def xhat(X: np.ndarray, modes, k: int) -> np.ndarray:
    """X reshaped to (I_1..I_{k-1}) x I_k x (I_{k+1}..I_m), k = 1..m."""
    P = int(np.prod(modes[: k - 1]))
    J = int(np.prod(modes[k:]))
    return np.asarray(X, dtype=np.float64).reshape(P, modes[k - 1], J, order="F")


def local_solve(A: np.ndarray, X3: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Eq. (5): G~ = A^T x_1 X^ x_3 B^T, returned as r_{k-1} x I_k x r_k."""
    P, n, J = X3.shape
    T = A.T @ X3.reshape(P, n * J, order="F")            # r_{k-1} x (I_k J)
    G = T.reshape(A.shape[1] * n, J, order="F") @ B.T    # (r_{k-1} I_k) x r_k
    return G.reshape(A.shape[1], n, B.shape[0], order="F")


def local_objective(A: np.ndarray, G: np.ndarray, B: np.ndarray, X3: np.ndarray) -> float:
    """Eq. (3)/(4): f(G) = 1/2 || X^ - A x G x B ||_F^2."""
    P, n, J = X3.shape
    approx = (A @ right_unfold(G)).reshape(P * n, G.shape[2], order="F") @ B
    d = X3.reshape(P * n, J, order="F") - approx
    return 0.5 * float(np.sum(d * d))


def reconstruct(cores, g) -> np.ndarray:
    """Slice reconstructed from a decomposition: G_1 x ... x G_m x g, shape (I_1..I_m)."""
    A = np.ones((1, 1))
    for G in cores:
        A = next_left_interface(A, G)
    modes = [G.shape[1] for G in cores]
    return (A @ np.asarray(g, dtype=np.float64)).reshape(modes, order="F")


def online_step(cores, g, X, *, instrument: bool = False, keep: bool = False,
                qr: Callable = householder_qr, lq: Callable = _lq,
                right_orth: bool = True, propagate: bool = True):
    """One Online TT-ALS update with slice X.  Returns (cores, g, StepInfo).

    right_orth=False and a different qr/lq exist only for tests of the
    method's invariances; the method itself is the default."""
    modes = [G.shape[1] for G in cores]
    m = len(cores)
    X = np.asarray(X, dtype=np.float64).reshape(modes, order="F")
    info = StepInfo(g_norm_in=float(np.linalg.norm(g)))

    # 1. right-orthogonalisation
    if right_orth:
        cores, g, _ = right_orthogonalize(cores, g, lq=lq)
    else:
        cores, g = copy_state(cores, g)
        cores, g, _ = normalize_g(cores, g)
    if keep:
        info.right_cores = [c.copy() for c in cores]

    # 2. right interfaces from the time t-1 cores
    B = right_interfaces(cores, g)

    # 3. forward update and left-orthogonalisation
    A = np.ones((1, 1))
    As, Gts = [A], []
    for k in range(1, m + 1):
        X3 = xhat(X, modes, k)
        Gt = local_solve(A, X3, B[k - 1])
        if instrument:
            info.f_before.append(local_objective(A, cores[k - 1], B[k - 1], X3))
            info.f_after.append(local_objective(A, Gt, B[k - 1], X3))
        Q, R = qr(left_unfold(Gt))
        cores[k - 1] = fold(Q, Gt.shape)
        if propagate:
            if k < m:
                nxt = cores[k]
                cores[k] = fold(R @ right_unfold(nxt), nxt.shape)
            else:
                g = R @ g
        A = next_left_interface(A, cores[k - 1])
        As.append(A)
        Gts.append(Gt)

    # 4. temporal row
    x = X.reshape(-1, order="F")
    g = A.T @ x
    M = (A @ g).reshape(modes, order="F")
    info.M = M
    info.E = float(np.linalg.norm(x - M.reshape(-1, order="F")))
    info.Xnorm = float(np.linalg.norm(x))
    info.f_final = 0.5 * info.E ** 2
    if keep:
        info.B, info.A, info.Gtilde = B, As, Gts
    return cores, g, info


@dataclass
class StreamResult:
    E: np.ndarray          # per-slice ||X_t - M_t||_F
    Xnorm: np.ndarray      # per-slice ||X_t||_F
    cores: list
    g: np.ndarray
    infos: list

    @property
    def re_per_slice(self) -> np.ndarray:
        return self.E / np.where(self.Xnorm > 0, self.Xnorm, 1.0)

    @property
    def re(self) -> float:
        """RE of the whole reconstructed stream (Section 5.1)."""
        return float(np.sqrt(np.sum(self.E ** 2) / np.sum(self.Xnorm ** 2)))


def run_stream(slices, cores0, g0, *, instrument=False, keep_M=False, **kw) -> StreamResult:
    """Apply the update to each slice in turn; slice t is reconstructed from
    the time-t decomposition (the output sequence of Algorithm 1)."""
    cores, g = copy_state(cores0, g0)
    check_ranks([c.shape[1] for c in cores], [c.shape[2] for c in cores])
    E, Xn, infos = [], [], []
    for X in slices:
        cores, g, info = online_step(cores, g, X, instrument=instrument, **kw)
        E.append(info.E)
        Xn.append(info.Xnorm)
        if not keep_M:
            info.M = None
        infos.append(info)
    return StreamResult(np.array(E), np.array(Xn), cores, g, infos)
