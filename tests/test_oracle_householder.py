"""Pins for the oracle's thin Householder QR / LQ (Algorithm 1's QR and LQ).

Checks: the factorisation reproduces its input, Q has orthonormal columns, R
is upper triangular with a non-negative diagonal, the result equals LAPACK's
QR (numpy) up to the sign convention, and rank-deficient inputs still give an
orthonormal Q (the oracle's completion rule)."""

import numpy as np
import pytest

from oracle.householder import householder_qr, lq


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


@pytest.mark.parametrize("m,n", [(1, 1), (5, 1), (8, 8), (32, 4), (72, 32), (480, 32), (33, 17)])
def test_qr_factorises_and_orthonormal(m, n):
    M = _rng(m * 100 + n).standard_normal((m, n))
    Q, R = householder_qr(M)
    assert Q.shape == (m, n) and R.shape == (n, n)
    assert np.linalg.norm(Q @ R - M) <= 1e-13 * np.linalg.norm(M)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13
    assert np.allclose(R, np.triu(R), atol=0)
    assert np.all(np.diag(R) >= 0)


@pytest.mark.parametrize("m,n", [(10, 3), (64, 32), (300, 16)])
def test_qr_matches_lapack_up_to_signs(m, n):
    M = _rng(7 + m).standard_normal((m, n))
    Q, R = householder_qr(M)
    Qn, Rn = np.linalg.qr(M)
    s = np.sign(np.diag(Rn))
    Qn, Rn = Qn * s[None, :], Rn * s[:, None]
    assert np.max(np.abs(Q - Qn)) <= 1e-12
    assert np.max(np.abs(R - Rn)) <= 1e-12 * np.max(np.abs(Rn))


@pytest.mark.parametrize("m,n,rank", [(96, 32, 1), (480, 32, 3), (32, 32, 1), (40, 8, 5)])
def test_qr_rank_deficient(m, n, rank):
    rng = _rng(m + n + rank)
    M = rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n))
    Q, R = householder_qr(M)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-13
    assert np.linalg.norm(Q @ R - M) <= 1e-12 * np.linalg.norm(M)
    # range(M) is contained in the span of Q's first `rank` columns
    P = Q[:, :rank] @ Q[:, :rank].T
    assert np.linalg.norm(P @ M - M) <= 1e-12 * np.linalg.norm(M)
    # the remaining diagonal of R is (numerically) zero
    assert np.all(np.abs(np.diag(R)[rank:]) <= 1e-12 * np.linalg.norm(M))


def test_qr_zero_matrix_gives_identity_columns():
    Q, R = householder_qr(np.zeros((7, 3)))
    assert np.array_equal(Q, np.eye(7, 3))
    assert np.array_equal(R, np.zeros((3, 3)))


@pytest.mark.parametrize("m,n", [(4, 128), (16, 48), (8, 288), (32, 32), (3, 3)])
def test_lq(m, n):
    M = _rng(m * n).standard_normal((m, n))
    L, Q = lq(M)
    assert np.linalg.norm(L @ Q - M) <= 1e-13 * np.linalg.norm(M)
    assert np.linalg.norm(Q @ Q.T - np.eye(m)) <= 1e-13
    assert np.allclose(L, np.tril(L), atol=0)
    assert np.all(np.diag(L) >= 0)


def test_qr_rejects_wide():
    with pytest.raises(ValueError):
        householder_qr(np.ones((2, 3)))
