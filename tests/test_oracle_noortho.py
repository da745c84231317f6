"""Pins of the "w/o Ortho" ablation oracle (oracle/noortho.py).

In exact arithmetic the ablation projects every slice onto the same spaces
as the proposed method (the row spaces of the right interfaces do not depend
on their gauge), so on short streams its reconstructions equal the pinned
main oracle's; its local solve equals a brute-force least-squares solution of
the local problem; the pseudo-inverse of the Gram matrix is numpy's; and its
right cores are not right-orthogonal."""

import numpy as np
import pytest

from oracle import noortho, ttals
from ttgen import exact_tt_stream

CASES = [((32, 32), (4, 4)), ((20, 18, 3), (6, 6, 3)), ((6, 5, 4, 3), (3, 4, 4, 2)), ((9,), (4,))]


@pytest.mark.parametrize("modes,ranks", CASES)
def test_reconstructions_equal_proposed_method(modes, ranks):
    st = exact_tt_stream(modes, ranks, ranks, 8, 41, 42, sigma=1e-2)
    init = st.init()
    xs = list(st.frames(1, st.T))
    a = ttals.run_stream(xs, init[0], init[1], keep_M=True)
    b = noortho.run_stream_noortho(xs, init[0], init[1], keep_M=True)
    for ia, ib, X in zip(a.infos, b.infos, xs):
        assert np.linalg.norm(ia.M - ib.M) <= 1e-8 * np.linalg.norm(X)


@pytest.mark.parametrize("J", [6, 2])
def test_local_solve_is_least_squares(J):
    rng = np.random.Generator(np.random.PCG64(5 + J))
    P, n, r0, r1 = 7, 3, 2, 3
    A, _ = np.linalg.qr(rng.standard_normal((P, r0)))          # orthonormal left interface
    B = rng.standard_normal((r1, J))
    X3 = rng.standard_normal((P, n, J))
    G = noortho.local_solve_gram(A, X3, B)
    # brute force: vec(A G_i B) for every slice i of the middle mode
    for i in range(n):
        K = np.kron(B.T, A)                       # vec(A Gi B) = (B^T kron A) vec(Gi)
        gi, *_ = np.linalg.lstsq(K, X3[:, i, :].reshape(-1, order="F"), rcond=None)
        assert np.allclose(G[:, i, :].reshape(-1, order="F"), gi, atol=1e-9)


def test_right_cores_are_not_right_orthogonal():
    st = exact_tt_stream((20, 18, 3), (6, 6, 3), (6, 6, 3), 3, 51, 52, sigma=1e-2)
    init = st.init()
    cores, g = init
    for X in st.frames(1, 3):
        cores, g, _ = noortho.online_step_noortho(cores, g, X)
    Rt = ttals.right_unfold(cores[1])
    assert np.linalg.norm(Rt @ Rt.T - np.eye(Rt.shape[0])) > 1e-3
    assert abs(np.linalg.norm(g) - 1.0) > 1e-3


def test_dropping_the_forward_qr_is_caught():
    """A planted mistake (the forward QR left out as well) breaks the pin."""
    st = exact_tt_stream((20, 18, 3), (6, 6, 3), (6, 6, 3), 3, 61, 62, sigma=1e-2)
    init = st.init()
    xs = list(st.frames(1, 3))
    a = ttals.run_stream(xs, init[0], init[1], keep_M=True)
    cores, g = init
    worst = 0.0
    for X, ia in zip(xs, a.infos):
        cores, g, ib = noortho.online_step_noortho(cores, g, X, qr=lambda M: (M, np.eye(M.shape[1])))
        worst = max(worst, float(np.linalg.norm(ia.M - ib.M) / np.linalg.norm(X)))
    assert worst > 1e-3


@pytest.mark.parametrize("r,J", [(4, 9), (6, 3), (5, 1), (3, 3)])
def test_right_gram_pinv_is_the_pseudo_inverse(r, J):
    B = np.random.Generator(np.random.PCG64(r * 10 + J)).standard_normal((r, J))
    assert np.allclose(noortho.right_gram_pinv(B), np.linalg.pinv(B @ B.T), atol=1e-10)
