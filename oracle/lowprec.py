"""Reduced-precision slice contractions (oracle; test infrastructure only).

The precision study (Section 3.4.2's remark on low precision; the BF16
contraction variant) rounds both operands of the two slice contractions
(Eq. 5 reassociated at the split point: Z = X B^T and Y = A^T X) to bfloat16
and accumulates in FP32.  The reference here is the exact definition: the
operands rounded to bfloat16, then multiplied and summed in FP64, so that any
FP32-accumulated result differs from it only by its accumulation error.

bfloat16 keeps the FP32 sign and exponent and the top 7 fraction bits; the
rounding is to nearest, ties to even (IEEE 754 round-to-nearest-even applied
at bit 16 of the FP32 encoding).  FP64 inputs are first rounded to FP32.
"""

from __future__ import annotations

import numpy as np


def round_fp32(x) -> np.ndarray:
    """IEEE round-to-nearest-even FP64 -> FP32 (values returned as FP64)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even), after rounding to FP32;
    values returned as FP64.  NaN stays NaN; overflow gives +-inf."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (rounded & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def pass1_bf16(X: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Z = rnd(X) rnd(B)^T in FP64: X is P x J, B is r x J."""
    return round_bf16(X) @ round_bf16(B).T


def pass2_bf16(X: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Y = rnd(A)^T rnd(X) in FP64: X is P x J, A is P x r."""
    return round_bf16(A).T @ round_bf16(X)


def accumulation_bound(Xr: np.ndarray, Wr: np.ndarray, terms: int, transpose_left: bool) -> np.ndarray:
    """Elementwise bound on the error of summing `terms` products in FP32
    (Higham's gamma_n = n u / (1 - n u), u = 2^-24) times the sum of the
    absolute products: |X| |W|^T (pass 1) or |W|^T |X| (pass 2)."""
    u = 2.0 ** -24
    gamma = terms * u / (1.0 - terms * u)
    if transpose_left:
        return gamma * (np.abs(Wr).T @ np.abs(Xr))
    return gamma * (np.abs(Xr) @ np.abs(Wr).T)
