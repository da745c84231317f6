"""tt_kernel_pass1_noalloc (include/tt_kernels.h): pass 1 with its partial
tiles in the library's static per-GPU scratch array instead of a caller
workspace.  Two calls in a row, the second with a smaller input (the array
keeps the first call's contents), each compared with tt_kernel_pass1 on the
same operands (bit for bit: same kernels and plan) and with a float64 NumPy
contraction of the same FP32-rounded operands (the kernel tests' bound); a
shape whose partial tiles exceed the array is refused before any launch."""

import numpy as np
import pytest

from tests.gpu_util import say, torch_cuda

pytestmark = pytest.mark.gpu


def _operands(torch, P, J, r, seed, tdt):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((P, J))
    B = rng.standard_normal((r, J)).astype(np.float32)
    Xd = torch.from_numpy(np.asfortranarray(X).reshape(-1, order="F").copy()).cuda().to(tdt)
    Bd = torch.from_numpy(np.asfortranarray(B).reshape(-1, order="F").copy()).cuda()
    return X, B, Xd, Bd


def _reference(torch, X, B, tdt):
    if tdt == torch.bfloat16:
        Xr = torch.from_numpy(X).to(torch.bfloat16).to(torch.float64).numpy()
    else:
        Xr = X.astype(np.float32).astype(np.float64)
    Bd = B.astype(np.float64)
    return Xr @ Bd.T, np.abs(Xr) @ np.abs(Bd).T


def test_noalloc_pass1_equals_the_workspace_entry_point_on_two_calls():
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    # a config-3-sized slice first, then a smaller one (ragged tiles)
    for call, (P, J, r, tdt) in enumerate([(1080, 5760, 32, torch.float32), (90, 70, 16, torch.float32),
                                           (200, 300, 48, torch.bfloat16)]):
        say(f"pass1_noalloc call {call}: P={P} J={J} r={r} {tdt}")
        X, B, Xd, Bd = _operands(torch, P, J, r, 9000 + call, tdt)
        Z0 = torch.full((P * r,), float("nan"), dtype=torch.float64, device="cuda")
        Z1 = torch.full((P * r,), float("nan"), dtype=torch.float64, device="cuda")
        f0 = torch.zeros(1, dtype=torch.int32, device="cuda")
        f1 = torch.zeros(1, dtype=torch.int32, device="cuda")
        ws = torch.empty(binding.tt_kernel_pass1_workspace(P, J, r), dtype=torch.uint8, device="cuda")
        assert binding.tt_kernel_pass1_workspace(P, J, r) <= binding.tt_kernel_pass1_noalloc_max()
        assert binding.tt_kernel_pass1(Xd, P, J, r, Bd, Z0, ws, f0) == 0
        assert binding.tt_kernel_pass1_noalloc(Xd, P, J, r, Bd, Z1, f1) == 0
        torch.cuda.synchronize()
        z0, z1 = Z0.cpu().numpy(), Z1.cpu().numpy()
        assert np.array_equal(z0, z1), call
        ref, bound = _reference(torch, X, B, tdt)
        Z = z1.reshape(P, r, order="F")
        assert np.all(np.abs(Z - ref) <= 2e-6 * bound + 1e-30), call
        assert int(f1.item()) == 0


def test_noalloc_pass1_refuses_a_shape_beyond_its_scratch():
    torch = torch_cuda()
    from paper_2606_31061_amd import binding
    P, J, r = 1 << 20, 1024, 64
    assert binding.tt_kernel_pass1_workspace(P, J, r) > binding.tt_kernel_pass1_noalloc_max()
    say("pass1_noalloc: oversized shape is refused on the host")
    x = torch.zeros(1, dtype=torch.float32, device="cuda")   # never read: refused before any launch
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = binding.tt_kernel_pass1_noalloc(x, P, J, r, x, x, flag)
    assert st == binding.TT_ERR_UNSUPPORTED
    assert b"32 MiB" in binding.load_library().tt_last_error_string()
