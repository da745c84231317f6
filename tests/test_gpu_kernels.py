"""Kernel-level parity of the update's building blocks, called through the C
ABI (include/tt_kernels.h): pass 1 and pass 2 against a float64 NumPy
contraction of the same FP32-rounded operands, and the FP64 Householder QR
against the oracle's QR and its defining properties."""

import numpy as np
import pytest

from oracle.householder import householder_qr
from tests.gpu_util import say, torch_cuda

pytestmark = pytest.mark.gpu


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


# The FP32 pass 2 runs k_pass2g where 4 <= P <= 1280 and r <= 32, with 1, 2,
# 4, 8 or 16 waves per column tile as P grows past 80, 160, 320 and 640 rows,
# 16-byte loads where P % 4 == 0 and 4-byte loads otherwise.  Its edges here:
# P % 8 == 4, P = 1280 with ten k-steps per wave, P = 4, odd P up to 1279,
# ranks and columns that leave part of a tile or of a block's tiles empty.
# k_pass2 runs elsewhere (P > 1280, r > 32, P < 4).
CASES = [(32, 32, 4), (240, 960, 16), (1080, 5760, 32), (100, 77, 5), (33, 1, 8), (200, 300, 48),
         (8, 777, 8), (4, 3, 1), (90, 70, 16), (6, 50, 3), (1090, 400, 40), (1084, 100, 32), (1280, 64, 32),
         (1284, 40, 7), (12, 33, 31), (600, 200, 20), (601, 300, 32), (161, 1000, 32), (2, 10, 3),
         (801, 50, 16), (97, 2000, 32), (1279, 70, 32), (1282, 40, 8)]


def _ref_round(X, dt):
    import torch
    if dt == torch.bfloat16:
        return torch.from_numpy(X).to(torch.bfloat16).to(torch.float64).numpy()
    return X.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("P,J,r", CASES)
@pytest.mark.parametrize("xdt", ["f32", "f64", "bf16"])
def test_pass1_matches_numpy(P, J, r, xdt):
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    say(f"pass1 P={P} J={J} r={r} {xdt}")
    rng = _rng(P * 7 + J + r)
    X = rng.standard_normal((P, J))
    B = rng.standard_normal((r, J)).astype(np.float32)
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[xdt]
    Xd = torch.from_numpy(np.asfortranarray(X).reshape(-1, order="F").copy()).cuda().to(tdt)
    Bd = torch.from_numpy(np.asfortranarray(B).reshape(-1, order="F").copy()).cuda()
    Zd = torch.full((P * r,), float("nan"), dtype=torch.float64, device="cuda")
    ws = torch.full((binding.tt_kernel_pass1_workspace(P, J, r),), 255, dtype=torch.uint8, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    for rep in range(2):  # the workspace needs no initialisation and can be reused
        assert binding.tt_kernel_pass1(Xd, P, J, r, Bd, Zd, ws, flag) == 0
        torch.cuda.synchronize()
        Z = Zd.cpu().numpy().reshape(P, r, order="F")
        Xr = _ref_round(X, tdt)
        ref = Xr @ B.astype(np.float64).T
        bound = np.abs(Xr) @ np.abs(B.astype(np.float64)).T
        assert np.all(np.abs(Z - ref) <= 2e-6 * bound + 1e-30), rep
    assert int(flag.item()) == 0


@pytest.mark.parametrize("P,J,r", CASES)
@pytest.mark.parametrize("xdt", ["f32", "f64", "bf16"])
def test_pass2_matches_numpy(P, J, r, xdt):
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    say(f"pass2 P={P} J={J} r={r} {xdt}")
    rng = _rng(P * 5 + J + r)
    X = rng.standard_normal((P, J))
    A = rng.standard_normal((P, r)).astype(np.float32)
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[xdt]
    Xd = torch.from_numpy(np.asfortranarray(X).reshape(-1, order="F").copy()).cuda().to(tdt)
    Ad = torch.from_numpy(np.asfortranarray(A).reshape(-1, order="F").copy()).cuda()
    Yd = torch.full((r * J,), float("nan"), dtype=torch.float64, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert binding.tt_kernel_pass2(Xd, P, J, r, Ad, Yd, flag) == 0
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy().reshape(r, J, order="F")
    Xr = _ref_round(X, tdt)
    ref = A.astype(np.float64).T @ Xr
    bound = np.abs(A.astype(np.float64)).T @ np.abs(Xr)
    assert np.all(np.abs(Y - ref) <= 2e-6 * bound + 1e-30)
    assert int(flag.item()) == 0


def test_passes_flag_nonfinite_slices():
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    say("pass flags nonfinite")
    P, J, r = 240, 960, 16
    X = np.ones((P, J))
    X[17, 300] = np.nan
    Xd = torch.from_numpy(X.reshape(-1, order="F").copy()).cuda().float()
    Bd = torch.ones(r * J, dtype=torch.float32, device="cuda")
    Ad = torch.ones(P * r, dtype=torch.float32, device="cuda")
    Zd = torch.zeros(P * r, dtype=torch.float64, device="cuda")
    Yd = torch.zeros(r * J, dtype=torch.float64, device="cuda")
    ws = torch.zeros(binding.tt_kernel_pass1_workspace(P, J, r), dtype=torch.uint8, device="cuda")
    f1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    f2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert binding.tt_kernel_pass1(Xd, P, J, r, Bd, Zd, ws, f1) == 0
    assert binding.tt_kernel_pass2(Xd, P, J, r, Ad, Yd, f2) == 0
    torch.cuda.synchronize()
    assert int(f1.item()) == 1 and int(f2.item()) == 1


QR_CASES = [(8, 8, None), (72, 32, None), (480, 32, None), (512, 32, None), (96, 32, 1), (480, 32, 3),
            (32, 32, 1), (5120, 16, None), (5120, 16, 3), (1, 1, None), (300, 7, None), (16, 16, 0),
            (513, 32, None), (7328, 32, None), (2049, 33, None), (4096, 32, 5), (1000, 1, None),
            (700, 48, None), (1500, 40, 7), (66, 40, None),
            # more than 64 columns: the reflector bit masks span several words
            (600, 100, None), (300, 130, 20), (160, 70, 66),
            # the first failing Cholesky pivot in the rows of the second, third and last of the
            # factorisation's four waves (and in the streamed path): the fallback must still run
            (72, 32, 12), (480, 32, 20), (512, 32, 28), (2000, 32, 17)]


@pytest.mark.parametrize("m,n,rank", QR_CASES)
def test_qr_matches_oracle(m, n, rank):
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    say(f"qr m={m} n={n} rank={rank}")
    rng = _rng(m * 31 + n)
    if rank is None:
        M = rng.standard_normal((m, n))
    elif rank == 0:
        M = np.zeros((m, n))
    else:
        M = rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n))
    Md = torch.from_numpy(M.T.copy()).cuda()      # (n, m) C-contiguous = m x n column-major
    Qd = torch.empty_like(Md)
    Rd = torch.empty((n, n), dtype=torch.float64, device="cuda")
    wk = torch.empty(m * n, dtype=torch.float64, device="cuda")
    assert binding.tt_kernel_qr(Md, Qd, Rd, wk) == 0
    torch.cuda.synchronize()
    Q = Qd.cpu().numpy().T
    R = Rd.cpu().numpy().T
    nrm = max(np.linalg.norm(M), 1e-300)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-12
    assert np.linalg.norm(Q @ R - M) <= 1e-12 * nrm
    assert np.allclose(R, np.triu(R), atol=0) and np.all(np.diag(R) >= 0)
    Qo, Ro = householder_qr(M)
    if rank is None:
        # full rank: the thin QR with diag(R) > 0 is unique
        assert np.max(np.abs(Q - Qo)) <= 1e-11
        assert np.max(np.abs(R - Ro)) <= 1e-11 * np.max(np.abs(Ro))
    else:
        # rank-deficient: the data columns agree; completions may differ
        k = max(rank, 0)
        if k:
            assert np.linalg.norm(Q[:, :k] @ Q[:, :k].T @ M - M) <= 1e-11 * nrm


@pytest.mark.parametrize("m,n,rank", [(32, 32, 1), (480, 32, 3), (300, 130, 20), (5120, 16, 3)])
def test_qr_without_r_gives_the_same_q(m, n, rank):
    """R = NULL skips the work that only R needs; Q must not change."""
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    say(f"qr without R m={m} n={n} rank={rank}")
    rng = _rng(m * 7 + n)
    M = rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n))
    Md = torch.from_numpy(M.T.copy()).cuda()
    Q1 = torch.empty_like(Md)
    Q2 = torch.empty_like(Md)
    Rd = torch.empty((n, n), dtype=torch.float64, device="cuda")
    wk = torch.empty(m * n, dtype=torch.float64, device="cuda")
    assert binding.tt_kernel_qr(Md, Q1, Rd, wk) == 0
    assert binding.tt_kernel_qr(Md, Q2, None, wk) == 0
    torch.cuda.synchronize()
    assert torch.equal(Q1, Q2)


@pytest.mark.parametrize("m,n,cond", [(3000, 32, 1e3), (3000, 32, 1e10), (700, 20, 1e10)])
def test_tall_qr_in_place_and_ill_conditioned(m, n, cond):
    """Tall matrices, Q overwriting M: a well-conditioned one takes the
    streamed CholeskyQR2, an ill-conditioned one fails its pivot test and
    falls back to Householder; both give an orthonormal Q and M = Q R."""
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    say(f"tall qr in place m={m} n={n} cond={cond:g}")
    rng = _rng(m + n)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    M = (U * np.logspace(0, -np.log10(cond), n)) @ V.T
    Md = torch.from_numpy(M.T.copy()).cuda()
    Rd = torch.empty((n, n), dtype=torch.float64, device="cuda")
    wk = torch.empty(m * n, dtype=torch.float64, device="cuda")
    assert binding.tt_kernel_qr(Md, Md, Rd, wk) == 0
    torch.cuda.synchronize()
    Q = Md.cpu().numpy().T
    R = Rd.cpu().numpy().T
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-12
    assert np.linalg.norm(Q @ R - M) <= 1e-12 * np.linalg.norm(M)
    assert np.all(np.diag(R) >= 0)
