"""BF16-input, FP32-accumulate contractions on the GPU.

Kernel level (include/tt_kernels.h): pass 1 and pass 2 against the exact
product of the BF16-rounded operands (oracle/lowprec.py), within the
worst-case FP32 accumulation bound, for every slice dtype, ragged shapes and
both rank tilings; the result is bitwise reproducible and the workspace is
reused without clearing.  Stream level: an update with BF16 contractions stays
within a stated distance of the FP64 oracle, and batches of BF16 streams are
bitwise equal to solo runs."""

import numpy as np
import pytest

from oracle import lowprec, ttals
from tests.gpu_util import rel, say, to_device_slice, torch_cuda
from ttgen import exact_tt_stream

pytestmark = pytest.mark.gpu

CASES = [(32, 32, 4), (240, 960, 16), (1080, 5760, 32), (100, 77, 5), (33, 1, 8), (200, 300, 48),
         (8, 777, 8), (4, 3, 1), (37, 53, 7), (1024, 129, 64), (72, 2000, 33)]


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _dev(torch, M, dt):
    return torch.from_numpy(np.asfortranarray(M).reshape(-1, order="F").copy()).cuda().to(dt)


@pytest.mark.parametrize("P,J,r", CASES)
@pytest.mark.parametrize("xdt", ["bf16", "f32", "f64"])
def test_pass1_bf16_matches_rounded_product(P, J, r, xdt):
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    say(f"pass1_bf16 P={P} J={J} r={r} {xdt}")
    rng = _rng(P * 13 + J + r)
    X = rng.standard_normal((P, J))
    B = rng.standard_normal((r, J)).astype(np.float32)
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[xdt]
    Xd = _dev(torch, X, tdt)
    Xin = Xd.to(torch.float64).cpu().numpy().reshape(P, J, order="F")  # the values the kernel receives
    Bd = _dev(torch, B, torch.float32)
    Zd = torch.full((P * r,), float("nan"), dtype=torch.float64, device="cuda")
    ws = torch.zeros(binding.tt_kernel_pass1_bf16_workspace(P, J, r), dtype=torch.uint8, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref = lowprec.pass1_bf16(Xin, B.astype(np.float64))
    bound = lowprec.accumulation_bound(lowprec.round_bf16(Xin), lowprec.round_bf16(B), J, transpose_left=False)
    prev = None
    for rep in range(2):
        assert binding.tt_kernel_pass1_bf16(Xd, P, J, r, Bd, Zd, ws, flag) == 0
        torch.cuda.synchronize()
        Z = Zd.cpu().numpy().reshape(P, r, order="F")
        assert np.all(np.abs(Z - ref) <= bound + 1e-300), rep
        if prev is not None:
            assert np.array_equal(Z, prev)
        prev = Z.copy()
    assert int(flag.item()) == 0


@pytest.mark.parametrize("P,J,r", CASES)
@pytest.mark.parametrize("xdt", ["bf16", "f32", "f64"])
def test_pass2_bf16_matches_rounded_product(P, J, r, xdt):
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    say(f"pass2_bf16 P={P} J={J} r={r} {xdt}")
    rng = _rng(P * 17 + J + 3 * r)
    X = rng.standard_normal((P, J))
    A = rng.standard_normal((P, r)).astype(np.float32)
    tdt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[xdt]
    Xd = _dev(torch, X, tdt)
    Xin = Xd.to(torch.float64).cpu().numpy().reshape(P, J, order="F")
    Ad = _dev(torch, A, torch.float32)
    Yd = torch.full((r * J,), float("nan"), dtype=torch.float64, device="cuda")
    ws = torch.zeros(binding.tt_kernel_pass2_bf16_workspace(P, J, r), dtype=torch.uint8, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref = lowprec.pass2_bf16(Xin, A.astype(np.float64))
    bound = lowprec.accumulation_bound(lowprec.round_bf16(Xin), lowprec.round_bf16(A), P, transpose_left=True)
    prev = None
    for rep in range(2):
        assert binding.tt_kernel_pass2_bf16(Xd, P, J, r, Ad, Yd, ws, flag) == 0
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy().reshape(r, J, order="F")
        assert np.all(np.abs(Y - ref) <= bound + 1e-300), rep
        if prev is not None:
            assert np.array_equal(Y, prev)
        prev = Y.copy()
    assert int(flag.item()) == 0


@pytest.mark.parametrize("which", ["pass1", "pass2"])
def test_bf16_pass_flags_nonfinite(which):
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    P, J, r = 240, 960, 16
    say(f"{which}_bf16 non-finite flag")
    rng = _rng(5)
    X = rng.standard_normal((P, J)).astype(np.float32)
    X[17, 400] = np.inf
    Xd = _dev(torch, X, torch.float32)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    if which == "pass1":
        W = _dev(torch, rng.standard_normal((r, J)).astype(np.float32), torch.float32)
        out = torch.zeros(P * r, dtype=torch.float64, device="cuda")
        ws = torch.zeros(binding.tt_kernel_pass1_bf16_workspace(P, J, r), dtype=torch.uint8, device="cuda")
        assert binding.tt_kernel_pass1_bf16(Xd, P, J, r, W, out, ws, flag) == 0
    else:
        W = _dev(torch, rng.standard_normal((P, r)).astype(np.float32), torch.float32)
        out = torch.zeros(r * J, dtype=torch.float64, device="cuda")
        ws = torch.zeros(binding.tt_kernel_pass2_bf16_workspace(P, J, r), dtype=torch.uint8, device="cuda")
        assert binding.tt_kernel_pass2_bf16(Xd, P, J, r, W, out, ws, flag) == 0
    torch.cuda.synchronize()
    assert int(flag.item()) == 1


# RE distance allowed between BF16 contractions and the FP64 oracle.  Rounding
# a slice to BF16 perturbs each entry by at most 2^-9 relative (RMS about
# 2^-9 / sqrt(3) = 1.1e-3), and a rank-r projection keeps only a small part of
# that perturbation, so the reconstruction error moves by well under 2e-3 of
# ||X||; the bound leaves a margin for the interface rounding.
RE_TOL_BF16 = 3e-3


@pytest.mark.parametrize("case", ["order3_32x32_r4", "order4_60x80x3_r8"])
def test_bf16_stream_tracks_oracle(case):
    torch = torch_cuda()
    from paper_2606_31061_amd import TTStream
    if case == "order3_32x32_r4":
        st = exact_tt_stream((32, 32), (4, 4), (4, 4), 30, 1001, 2001, sigma=1e-3)
    else:
        st = exact_tt_stream((60, 80, 3), (8, 8, 3), (8, 8, 3), 20, 1002, 2002, sigma=1e-2)
    init = st.init()
    xs = list(st.frames(1, st.T))
    say(f"bf16 stream {case}")
    s = TTStream(st.modes, st.ranks, init=init, compute="bf16")
    res = ttals.run_stream(xs, init[0], init[1])
    E = []
    for X in xs:
        s.push(to_device_slice(torch, X.astype(np.float32), torch.bfloat16))
        M = s.reconstruct()
        E.append(np.linalg.norm(X - M))
    s.synchronize()
    re_gpu = float(np.sqrt(np.sum(np.square(E)) / np.sum(np.square(res.Xnorm))))
    assert abs(re_gpu - res.re) <= RE_TOL_BF16, (re_gpu, res.re)
    # the gauge cores stay orthogonal (FP64 QR)
    cores, g, t = s.get_state()
    assert t == len(xs)
    for G in cores[:-1]:
        L = ttals.left_unfold(G)
        assert np.linalg.norm(L.T @ L - np.eye(L.shape[1])) <= 1e-10
    s.close()


def test_bf16_batch_bitwise_equal_to_solo():
    torch = torch_cuda()
    from paper_2606_31061_amd import TTBatch, TTStream
    T = 4
    sts = [exact_tt_stream((40, 36, 3), (6, 6, 3), (6, 6, 3), T, 700 + q, 800 + q, sigma=1e-2) for q in range(3)]
    say("bf16 batch of 3 (40,36,3)")
    solo, members = [], []
    for st in sts:
        init = st.init()
        solo.append(TTStream(st.modes, st.ranks, init=init, compute="bf16"))
        members.append(TTStream(st.modes, st.ranks, init=init, compute="bf16"))
    batch = TTBatch(members)
    dev = [[to_device_slice(torch, X, torch.bfloat16) for X in st.frames(1, T)] for st in sts]
    for t in range(T):
        for s, xs in zip(solo, dev):
            s.push(xs[t])
        batch.push([xs[t] for xs in dev])
    assert batch.synchronize() == [0, 0, 0]
    for a, b in zip(solo, members):
        ca, ga, ta = a.get_state()
        cb, gb, tb = b.get_state()
        assert ta == tb == T
        assert all(np.array_equal(x, y) for x, y in zip(ca, cb)) and np.array_equal(ga, gb)
    batch.close()
