"""Helpers shared by the GPU tests (device setup and stream runners)."""

import sys

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def say(msg: str) -> None:
    """Name the case on stdout before a GPU step (survives a crash of the step)."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def to_device_slice(torch, X: np.ndarray, dtype=None):
    """Device copy of slice X with i_1 fastest (flat)."""
    flat = np.ascontiguousarray(np.asarray(X).reshape(-1, order="F"))
    t = torch.from_numpy(flat).cuda()
    if dtype is not None:
        t = t.to(dtype)
    return t


def run_gpu_stream(torch, modes, ranks, init, slices, *, recon_every=True, split_point=0, dtype=None):
    """Push every slice; return per-slice reconstructions (or None) and the handle."""
    from paper_2606_31061_amd import TTStream
    s = TTStream(modes, ranks, init=init, split_point=split_point, keep_history=True, history_capacity=4096)
    Ms = []
    for X in slices:
        s.push(to_device_slice(torch, X, dtype))
        if recon_every:
            Ms.append(s.reconstruct())
    s.synchronize()
    return Ms, s


def rel(a, b, scale) -> float:
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) / scale)
