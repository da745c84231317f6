"""The oracle's pins catch plausible mistakes.

Each test plants one mistake in the oracle (monkeypatched, CPU only) and checks
that a pin which passes on the correct oracle fails on the mutated one: a
transposed reshape, a wrong-side absorption in the LQ sweep, a reflector
missing its factor 2, a transposed R propagation, a perturbed interface, and
a dropped normalisation."""

import numpy as np
import pytest

from oracle import ttals, closed_form, householder
from ttgen import config_c1, exact_tt_stream


def _c1():
    s = config_c1(T=12)
    cores, g = s.init()
    return list(s.frames(1, 12)), cores, g


def _closed_form_err(slices, cores, g):
    res = ttals.run_stream(slices, cores, g, keep_M=True)
    return max(np.linalg.norm(i.M - Mc) / np.linalg.norm(X)
               for i, Mc, X in zip(res.infos, closed_form.order3_outputs(slices, cores[1], g), slices))


def _order4():
    s = exact_tt_stream((6, 5, 4, 3), (3, 4, 4, 2), (3, 4, 4, 2), 6, 11, 12, sigma=0.0)
    cores, g = s.init()
    return list(s.frames(1, 6)), cores, g


def _exact_recovery_err(slices, cores, g):
    return float(np.max(ttals.run_stream(slices, cores, g).re_per_slice))


def test_baseline_pins_pass():
    assert _closed_form_err(*_c1()) <= 1e-12
    assert _exact_recovery_err(*_order4()) <= 1e-12


def test_transposed_reshape_is_caught(monkeypatch):
    def bad_xhat(X, modes, k):
        P = int(np.prod(modes[: k - 1]))
        J = int(np.prod(modes[k:]))
        return np.asarray(X, dtype=np.float64).reshape(P, modes[k - 1], J, order="C")
    monkeypatch.setattr(ttals, "xhat", bad_xhat)
    assert _exact_recovery_err(*_order4()) > 1e-3


def test_absorbing_L_transposed_is_caught(monkeypatch):
    real_lq = householder.lq

    def bad_lq(M, tol=householder.DEFAULT_TOL):
        L, Q = real_lq(M, tol)
        return L.T, Q
    s = exact_tt_stream((6, 5, 4), (3, 4, 2), (3, 4, 2), 4, 1, 2, sigma=1e-2)
    cores, g = s.init()
    X = s.frame(1)
    c, gg, _ = ttals.online_step(cores, g, X)
    before = ttals.reconstruct(c, gg)
    rc, rg, _ = ttals.right_orthogonalize(c, gg, lq=bad_lq)
    assert np.linalg.norm(ttals.reconstruct(rc, rg) - before) > 1e-6 * np.linalg.norm(before)


def test_reflector_without_factor_two_is_caught(monkeypatch):
    def bad_qr(M, tol=householder.DEFAULT_TOL):
        A = np.array(M, dtype=np.float64)
        m, n = A.shape
        Q = np.eye(m)[:, :n].copy()
        for j in range(n):
            x = A[j:, j]
            v = x.copy()
            v[0] += np.linalg.norm(x) * (1 if x[0] >= 0 else -1)
            A[j:, j:] -= np.outer(v, (1.0 / (v @ v)) * (v @ A[j:, j:]))
        return np.linalg.qr(M)[0], np.triu(A[:n])
    M = np.random.Generator(np.random.PCG64(1)).standard_normal((20, 5))
    Q, R = bad_qr(M)
    assert np.linalg.norm(Q @ R - M) > 1e-3 * np.linalg.norm(M)
    Qg, Rg = householder.householder_qr(M)
    assert np.linalg.norm(Qg @ Rg - M) <= 1e-13 * np.linalg.norm(M)


def test_transposed_r_propagation_is_caught():
    """Propagating R^T instead of R leaves M_t (the propagated core is
    overwritten) but breaks the continuity f_k^before = f_{k-1}^after (P3)."""
    st = exact_tt_stream((6, 5, 4, 3), (3, 4, 4, 2), (3, 4, 4, 2), 3, 11, 12, sigma=5e-2)
    cores, g = st.init()
    X = st.frame(1)

    def qr_rt(M):
        Q, R = householder.householder_qr(M)
        return Q, R.T
    _, _, good = ttals.online_step(cores, g, X, instrument=True)
    _, _, bad = ttals.online_step(cores, g, X, instrument=True, qr=qr_rt)
    gap = lambda i: max(abs(i.f_before[k] - i.f_after[k - 1]) / i.f_before[0] for k in range(1, 4))
    assert gap(good) <= 1e-11
    assert gap(bad) > 1e-6
    assert np.linalg.norm(good.M - bad.M) <= 1e-11 * np.linalg.norm(X)


def test_interfaces_from_updated_cores_is_caught(monkeypatch):
    """Building B_k from the time-t cores (not t-1) changes the outputs."""
    slices, cores, g = _c1()
    real_solve = ttals.local_solve

    def bad_solve(A, X3, B):
        # replace B_1 by an interface built from a different (perturbed) core
        if A.shape == (1, 1):
            B = B + 0.5 * np.random.Generator(np.random.PCG64(0)).standard_normal(B.shape)
        return real_solve(A, X3, B)
    monkeypatch.setattr(ttals, "local_solve", bad_solve)
    assert _closed_form_err(slices, cores, g) > 1e-6


def test_dropped_normalisation_changes_nothing_but_is_seen_by_p1(monkeypatch):
    """Skipping the normalisation leaves M_t (gauge) but breaks ||g|| = 1 of P1."""
    slices, cores, g = _c1()
    monkeypatch.setattr(ttals, "normalize_g", lambda c, g: (c, g, 1.0))
    rc, rg, _ = ttals.right_orthogonalize(cores, g)
    assert abs(np.linalg.norm(rg) - 1.0) > 1e-3
