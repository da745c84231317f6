"""Pins of the FP64 oracle of Algorithm 1 against what the paper and the
mathematics fix (there is no worked example in the paper).

P1  orthogonality of the gauge cores (Section 2.4 definition, Algorithm 1)
P2  right-orthogonalisation preserves the represented slice (proof of Prop. 2)
P3  continuity of the local objective along the sweep (Eq. 3 with Algorithm 1)
P4  stationarity of the final least-squares step for g (Eq. 5 with B_n = 1)
P5  Proposition 1's identity f(old) - f(new) = 1/2 ||G_old - G_new||^2 when its
    hypothesis B_k B_k^T = I holds (r_{n-1} = 1)
P6  an r_{n-1} > 1 run equals the r_{n-1} = 1 run with matched initial cores
P7  the order-3 closed form (a cross-Gram subspace iteration)
P8  M_t is the projection of X_t onto the left interface of cores 1..m-1
P9  exact recovery of an exactly TT-rank-r stream
P10 Eckart-Young lower bound and the batch TT-SVD comparison
P11 outputs independent of the QR completion rule and of the gauge sweep
P12 Proposition 2 (temporal smoothness bound) when its hypothesis holds
"""

import numpy as np
import pytest

from oracle import ttals, closed_form, ttsvd, metrics
from oracle.householder import householder_qr
from ttgen import exact_tt_stream, config_c1, init_cores, tt_full


def _stream(modes, ranks, T=8, sigma=1e-3, data_seed=11, init_seed=12, true_ranks=None):
    true_ranks = true_ranks or ranks
    s = exact_tt_stream(modes, true_ranks, ranks, T, data_seed, init_seed, sigma=sigma)
    cores, g = s.init()
    return list(s.frames(1, T)), cores, g


SHAPES = [
    ((32, 32), (4, 4)),
    ((12, 10, 3), (4, 4, 4)),
    ((6, 5, 4, 3), (3, 4, 4, 2)),
    ((5, 1, 4, 1), (3, 3, 4, 4)),      # modes of size 1
    ((7, 6), (5, 1)),                   # r_{n-1} = 1
]


def _orth_err_left(G):
    L = ttals.left_unfold(G)
    return np.linalg.norm(L.T @ L - np.eye(L.shape[1]))


def _orth_err_right(G):
    R = ttals.right_unfold(G)
    return np.linalg.norm(R @ R.T - np.eye(R.shape[0]))


@pytest.mark.parametrize("modes,ranks", SHAPES)
def test_p1_orthogonality(modes, ranks):
    slices, cores, g = _stream(modes, ranks)
    rc, rg, _ = ttals.right_orthogonalize(cores, g)
    assert abs(np.linalg.norm(rg) - 1.0) <= 1e-14
    for k in range(1, len(rc)):
        assert _orth_err_right(rc[k]) <= 1e-12
    c, gg = cores, g
    for X in slices:
        c, gg, _ = ttals.online_step(c, gg, X)
        for G in c:
            assert _orth_err_left(G) <= 1e-12


@pytest.mark.parametrize("modes,ranks", SHAPES)
def test_p2_right_orth_preserves_slice(modes, ranks):
    slices, cores, g = _stream(modes, ranks)
    c, gg, _ = ttals.online_step(cores, g, slices[0])
    before = ttals.reconstruct(c, gg)
    rc, rg, nu = ttals.right_orthogonalize(c, gg)
    after = ttals.reconstruct(rc, rg)
    assert np.linalg.norm(after - before) <= 1e-12 * np.linalg.norm(before)


@pytest.mark.parametrize("modes,ranks", SHAPES)
def test_p3_objective_chain_continuity(modes, ranks):
    slices, cores, g = _stream(modes, ranks)
    c, gg = cores, g
    prev_M = ttals.reconstruct(ttals.right_orthogonalize(c, gg)[0], ttals.right_orthogonalize(c, gg)[1])
    for X in slices:
        c, gg, info = ttals.online_step(c, gg, X, instrument=True)
        scale = max(info.f_before[0], 1e-300)
        # f_1 before = 1/2 ||X_t - M_{t-1}||^2
        d = X - prev_M
        assert abs(info.f_before[0] - 0.5 * np.sum(d * d)) <= 1e-11 * scale
        for k in range(1, len(c)):
            assert abs(info.f_before[k] - info.f_after[k - 1]) <= 1e-11 * scale
        # the final least-squares step can only lower the objective
        assert info.f_final <= info.f_after[-1] * (1 + 1e-12) + 1e-300
        # at k = m the local solve is a minimiser (B_m = g has unit norm)
        assert info.f_after[-1] <= info.f_before[-1] * (1 + 1e-12) + 1e-300
        prev_M = info.M


@pytest.mark.parametrize("modes,ranks", SHAPES)
def test_p4_final_least_squares_stationarity(modes, ranks):
    slices, cores, g = _stream(modes, ranks)
    c, gg = cores, g
    for X in slices:
        c, gg, info = ttals.online_step(c, gg, X, keep=True)
        A = info.A[-1]
        x = X.reshape(-1, order="F")
        Mv = info.M.reshape(-1, order="F")
        assert np.linalg.norm(A.T @ (x - Mv)) <= 1e-12 * np.linalg.norm(x)
        assert abs(np.dot(x - Mv, Mv)) <= 1e-12 * np.dot(x, x)
        assert abs(np.linalg.norm(gg) - np.linalg.norm(Mv)) <= 1e-12 * np.linalg.norm(x)


@pytest.mark.parametrize("modes,ranks", [((7, 6), (5, 1)), ((12, 10, 3), (4, 3, 1)), ((6, 5, 4, 3), (3, 4, 3, 1))])
def test_p5_proposition1_identity_when_hypothesis_holds(modes, ranks):
    slices, cores, g = _stream(modes, ranks, sigma=1e-2)
    c, gg = cores, g
    for X in slices:
        c_in, g_in = c, gg
        c, gg, info = ttals.online_step(c, gg, X, instrument=True, keep=True)
        # hypothesis: B_k B_k^T = I for every k
        for B in info.B:
            assert np.linalg.norm(B @ B.T - np.eye(B.shape[0])) <= 1e-12
        # recompute the cores entering each local solve to measure ||G_old - G_new||
        rc, rg, _ = ttals.right_orthogonalize(c_in, g_in)
        cur = [x.copy() for x in rc]
        for k in range(len(cur)):
            Gt = info.Gtilde[k]
            lhs = info.f_before[k] - info.f_after[k]
            rhs = 0.5 * np.sum((cur[k] - Gt) ** 2)
            assert lhs >= -1e-12 * max(info.f_before[k], 1.0)
            assert abs(lhs - rhs) <= 1e-10 * max(info.f_before[k], 1e-300)
            Q, R = householder_qr(ttals.left_unfold(Gt))
            if k + 1 < len(cur):
                cur[k + 1] = ttals.fold(R @ ttals.right_unfold(cur[k + 1]), cur[k + 1].shape)


@pytest.mark.parametrize("modes,ranks", [((32, 32), (4, 4)), ((12, 10, 6), (4, 4, 4)), ((6, 5, 4, 3), (3, 4, 3, 3))])
def test_p6_temporal_rank_reduction(modes, ranks):
    slices, cores, g = _stream(modes, ranks, sigma=1e-2)
    c1 = [x.copy() for x in cores]
    last = c1[-1]
    c1[-1] = (ttals.left_unfold(last) @ g).reshape(last.shape[0], last.shape[1], 1, order="F")
    g1 = np.ones(1)
    ra = ttals.run_stream(slices, cores, g, keep_M=True)
    rb = ttals.run_stream(slices, c1, g1, keep_M=True)
    for ia, ib, X in zip(ra.infos, rb.infos, slices):
        assert np.linalg.norm(ia.M - ib.M) <= 1e-11 * np.linalg.norm(X)


def test_p7_order3_closed_form():
    s = config_c1(T=40)
    cores, g = s.init()
    slices = list(s.frames(1, 40))
    res = ttals.run_stream(slices, cores, g, keep_M=True)
    for info, Mc, X in zip(res.infos, closed_form.order3_outputs(slices, cores[1], g), slices):
        assert np.linalg.norm(info.M - Mc) <= 1e-12 * np.linalg.norm(X)


@pytest.mark.parametrize("modes,ranks", SHAPES)
def test_p8_projection_structure(modes, ranks):
    slices, cores, g = _stream(modes, ranks)
    c, gg = cores, g
    m = len(modes)
    for X in slices:
        c, gg, info = ttals.online_step(c, gg, X, keep=True)
        Am = info.A[m - 1]                          # A_m: left interface of cores 1..m-1
        Xm = X.reshape(Am.shape[0], -1, order="F")  # (I_1..I_{m-1}) x I_m
        P = Am @ (Am.T @ Xm)
        assert np.linalg.norm(P.reshape(X.shape, order="F") - info.M) <= 1e-12 * np.linalg.norm(X)
        # the temporal row is 1-sparse with magnitude ||M_t||
        nz = np.abs(gg) > 1e-12 * np.linalg.norm(gg)
        assert nz.sum() <= 1


@pytest.mark.parametrize("modes,ranks", SHAPES[:4] + [((8, 9, 15, 1, 3), (8, 16, 16, 16, 16))])
def test_p9_exact_recovery(modes, ranks):
    slices, cores, g = _stream(modes, ranks, T=6, sigma=0.0)
    res = ttals.run_stream(slices, cores, g)
    assert np.all(res.re_per_slice <= 1e-12)


def test_p10_eckart_young_lower_bound_and_ttsvd():
    for modes, ranks in [((32, 32), (4, 4)), ((12, 10, 3), (4, 4, 4))]:
        slices, cores, g = _stream(modes, ranks, T=30, sigma=1e-2, true_ranks=tuple(ranks))
        res = ttals.run_stream(slices, cores, g)
        m = len(modes)
        for X, E in zip(slices, res.E):
            for k in range(1, m):
                assert ttsvd.unfolding_tail(X, k, ranks[k - 1]) <= E * (1 + 1e-12)
        # batch TT-SVD of the stream at the same ranks.  Slice 1 is excluded
        # on both sides: its error reflects the random initial cores.
        full = np.stack(slices[1:], axis=-1)
        tcores, tails = ttsvd.tt_svd(full, list(ranks))
        re_b = metrics.relative_error(full, ttsvd.tt_to_full(tcores))
        re_o = metrics.stream_re(res.E[1:], res.Xnorm[1:])
        assert re_online_ratio_ok(re_o, re_b)
    # noise-free: both exact
    slices, cores, g = _stream((12, 10, 3), (4, 4, 4), T=12, sigma=0.0)
    res = ttals.run_stream(slices, cores, g)
    full = np.stack(slices, axis=-1)
    tcores, _ = ttsvd.tt_svd(full, [4, 4, 4])
    assert res.re <= 1e-12
    assert metrics.relative_error(full, ttsvd.tt_to_full(tcores)) <= 1e-12


def re_online_ratio_ok(re_online, re_batch, gate=3.0):
    return re_online <= gate * re_batch


def _random_completion_qr(seed):
    rng = np.random.Generator(np.random.PCG64(seed))

    def qr(M):
        Q, R = householder_qr(M)
        # replace the completion columns (zero diagonal of R) by a random
        # orthonormal completion; the factorisation Q R = M is unchanged
        dead = np.abs(np.diag(R)) <= 1e-12 * max(np.linalg.norm(M), 1e-300)
        if dead.any():
            live = Q[:, ~dead]
            C = rng.standard_normal((M.shape[0], int(dead.sum())))
            C -= live @ (live.T @ C)
            Qc, _ = np.linalg.qr(C)
            Qc -= live @ (live.T @ Qc)
            Qc, _ = np.linalg.qr(Qc)
            Q = Q.copy()
            Q[:, dead] = Qc
        return Q, R

    return qr


@pytest.mark.parametrize("modes,ranks", [((12, 10, 3), (4, 4, 4)), ((6, 5, 4, 3), (3, 4, 4, 2)), ((5, 1, 4, 1), (3, 3, 4, 4))])
def test_p11_completion_and_gauge_independence(modes, ranks):
    slices, cores, g = _stream(modes, ranks, T=10, sigma=1e-2)
    ref = ttals.run_stream(slices, cores, g, keep_M=True)
    alt = ttals.run_stream(slices, cores, g, keep_M=True, qr=_random_completion_qr(5))
    nosweep = ttals.run_stream(slices, cores, g, keep_M=True, right_orth=False)
    for a, b, c, X in zip(ref.infos, alt.infos, nosweep.infos, slices):
        assert np.linalg.norm(a.M - b.M) <= 1e-11 * np.linalg.norm(X)
        assert np.linalg.norm(a.M - c.M) <= 1e-11 * np.linalg.norm(X)


@pytest.mark.parametrize("modes,ranks", [((7, 6), (5, 1)), ((12, 10, 3), (4, 3, 1))])
def test_p12_proposition2_bound(modes, ranks):
    slices, cores, g = _stream(modes, ranks, T=20, sigma=5e-2)
    res = ttals.run_stream(slices, cores, g)
    for t in range(1, len(slices)):
        eps = np.linalg.norm(slices[t] - slices[t - 1])
        assert res.E[t] <= res.E[t - 1] + eps + 1e-12 * np.linalg.norm(slices[t])


def test_zero_slice_and_recovery():
    slices, cores, g = _stream((12, 10, 3), (4, 4, 4), T=6)
    slices[2] = np.zeros_like(slices[2])
    res = ttals.run_stream(slices, cores, g, keep_M=True)
    assert res.E[2] == 0.0 and np.all(res.infos[2].M == 0.0)
    assert res.infos[3].g_norm_in == 0.0          # normalisation falls back to e_1
    assert np.all(np.isfinite(res.E)) and res.re_per_slice[3] < 1.0


def test_order2_stream_is_exact():
    rng = np.random.Generator(np.random.PCG64(3))
    cores, g = init_cores((9,), (4,), 4)
    slices = [rng.standard_normal((9,)) for _ in range(4)]
    res = ttals.run_stream(slices, cores, g)
    assert np.all(res.re_per_slice <= 1e-14)


def test_clamp_ranks():
    assert ttals.clamp_ranks((8, 9, 15, 8, 16, 15, 3, 1, 1), [32] * 9) == [8] + [32] * 8
    assert ttals.clamp_ranks((32, 32), (4, 4)) == [4, 4]
    assert ttals.clamp_ranks((2, 2, 2), (8, 8, 8)) == [2, 4, 8]
    assert ttals.clamp_ranks((3, 1, 1), (5, 5, 2)) == [2, 2, 2]
    with pytest.raises(ValueError):
        ttals.check_ranks((2, 2), (4, 4))


def test_tt_svd_pins():
    rng = np.random.Generator(np.random.PCG64(9))
    # matrix case: TT-SVD is the truncated SVD, error equals the Eckart-Young tail
    M = rng.standard_normal((20, 15))
    tc, tails = ttsvd.tt_svd(M, [5])
    err = np.linalg.norm(M - ttsvd.tt_to_full(tc))
    s = np.linalg.svd(M, compute_uv=False)
    assert abs(err - np.sqrt(np.sum(s[5:] ** 2))) <= 1e-12 * np.linalg.norm(M)
    # exact TT-rank tensor is recovered
    cores = [rng.standard_normal(sh) for sh in [(1, 6, 3), (3, 5, 4), (4, 4, 2), (2, 3, 1)]]
    X = ttsvd.tt_to_full(cores)
    tc, tails = ttsvd.tt_svd(X, [3, 4, 2])
    assert np.linalg.norm(X - ttsvd.tt_to_full(tc)) <= 1e-12 * np.linalg.norm(X)
    # noisy tensor: the error lies between the largest unfolding tail and the bound
    Y = X + 0.05 * rng.standard_normal(X.shape)
    tc, tails = ttsvd.tt_svd(Y, [3, 4, 2])
    err = np.linalg.norm(Y - ttsvd.tt_to_full(tc))
    lower = max(ttsvd.unfolding_tail(Y, k, r) for k, r in zip([1, 2, 3], [3, 4, 2]))
    assert lower <= err * (1 + 1e-12)
    assert err <= np.sqrt(np.sum(np.square(tails))) * (1 + 1e-12)


def test_generator_tt_full_matches_definition():
    rng = np.random.Generator(np.random.PCG64(2))
    cores = [rng.standard_normal(sh) for sh in [(1, 3, 2), (2, 4, 3), (3, 2, 2)]]
    h = rng.standard_normal(2)
    X = tt_full(cores, h)
    ref = np.einsum("ia,ajb,bkc,c->ijk", cores[0][0], cores[1], cores[2], h)
    assert np.allclose(X, ref, atol=1e-14)
