"""Pins of the reduced-precision reference (oracle/lowprec.py): the bfloat16
rounding against worked values of the format's definition and against
PyTorch's own conversion (an independent implementation), and the BF16
contractions against exact products where rounding changes nothing."""

import numpy as np
import pytest

from oracle import lowprec


def test_round_bf16_worked_values():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert lowprec.round_bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 2^-8 is halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert lowprec.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    # just above the halfway point rounds up
    assert lowprec.round_bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert lowprec.round_bf16(-(1.0 + 2.0 ** -8)) == -1.0
    # representable values are unchanged
    for v in [0.0, -0.0, 1.0, -2.5, 0.15625, 2.0 ** -130, 3.0 * 2.0 ** 100]:
        assert lowprec.round_bf16(v) == lowprec.round_fp32(v)
    # the largest FP32 value rounds beyond the largest bfloat16 value
    assert np.isinf(lowprec.round_bf16(np.finfo(np.float32).max))
    assert np.isinf(lowprec.round_bf16(np.inf)) and np.isnan(lowprec.round_bf16(np.nan))
    # the largest bfloat16 value (2 - 2^-7) 2^127 is kept
    big = (2.0 - 2.0 ** -7) * 2.0 ** 127
    assert lowprec.round_bf16(big) == big


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.Generator(np.random.PCG64(7))
    x = np.concatenate([rng.standard_normal(20000) * s for s in (1e-40, 1e-3, 1.0, 1e5, 1e37)])
    # exact ties with both parities of the kept last bit
    base = rng.integers(0x3F800000, 0x40000000, size=5000, dtype=np.uint64)
    ties = ((base & ~np.uint64(0xFFFF)) | np.uint64(0x8000)).astype(np.uint32).view(np.float32)
    x = np.concatenate([x, ties.astype(np.float64)])
    mine = lowprec.round_bf16(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mine, ref)


def test_fp64_input_rounds_through_fp32():
    # a value just above a bfloat16 tie in FP64 that is a tie after rounding to FP32
    x = 1.0 + 2.0 ** -8 + 2.0 ** -40
    assert lowprec.round_fp32(x) == 1.0 + 2.0 ** -8
    assert lowprec.round_bf16(x) == 1.0


def test_bf16_contractions_exact_on_representable_operands():
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.integers(-8, 9, size=(40, 70)).astype(np.float64)
    B = rng.integers(-8, 9, size=(5, 70)).astype(np.float64)
    A = rng.integers(-8, 9, size=(40, 3)).astype(np.float64)
    assert np.array_equal(lowprec.pass1_bf16(X, B), X @ B.T)
    assert np.array_equal(lowprec.pass2_bf16(X, A), A.T @ X)


def test_accumulation_bound_covers_fp32_recursive_sum():
    rng = np.random.Generator(np.random.PCG64(11))
    X = lowprec.round_bf16(rng.standard_normal((6, 3000)))
    B = lowprec.round_bf16(rng.standard_normal((4, 3000)))
    exact = X @ B.T
    acc = np.zeros((6, 4), dtype=np.float32)
    for j in range(X.shape[1]):
        acc = (acc + np.outer(X[:, j], B[:, j]).astype(np.float32)).astype(np.float32)
    err = np.abs(acc.astype(np.float64) - exact)
    assert np.all(err <= lowprec.accumulation_bound(X, B, X.shape[1], transpose_left=False))
