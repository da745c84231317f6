"""ctypes binding of the C ABI (include/tt_stream.h, include/tt_kernels.h).

Argument marshalling only: every step of an update runs in the HIP library
lib/libttstream.so.  Device memory and streams come from PyTorch (ROCm build):
device tensors are passed by data_ptr() and streams by their hipStream_t.
Loading fails loudly when the library has not been built; there is no CPU
fallback.

The functions named like the C entry points (tt_stream_create, ...) map one to
one onto them; TTStream is a small convenience wrapper over the same calls.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t,
                    c_uint32, c_uint64, c_void_p)
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libttstream.so")

TT_OK, TT_ERR_INVALID_ARG, TT_ERR_SHAPE, TT_ERR_RANK, TT_ERR_OOM = 0, 1, 2, 3, 4
TT_ERR_DEVICE, TT_ERR_NONFINITE, TT_ERR_STATE, TT_ERR_UNSUPPORTED = 5, 6, 7, 8
STATUS_NAMES = {0: "TT_OK", 1: "TT_ERR_INVALID_ARG", 2: "TT_ERR_SHAPE", 3: "TT_ERR_RANK", 4: "TT_ERR_OOM",
                5: "TT_ERR_DEVICE", 6: "TT_ERR_NONFINITE", 7: "TT_ERR_STATE", 8: "TT_ERR_UNSUPPORTED"}
TT_F64, TT_F32, TT_BF16 = 0, 1, 2
TT_FLAG_SYNC_PUSH = 0x1
TT_FLAG_NO_ORTHO = 0x2
TT_FLAG_PROFILE_OPS = 0x4
TT_FLAG_AUTOTUNE = 0x8
TT_FLAG_WAVE_PLAN = 0x10


class TTError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class tt_allocator(Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", c_void_p)]


def make_allocator(alloc, free):
    """tt_allocator from Python callables alloc(nbytes) -> device pointer (int,
    0 on failure) and free(ptr).  The returned structure holds the ctypes
    callbacks; keep it alive as long as the handle that uses it."""
    a = ALLOC_FN(lambda n, ctx: int(alloc(int(n))) or None)
    f = FREE_FN(lambda p, ctx: free(int(p or 0)))
    st = tt_allocator(a, f, None)
    st._keep = (a, f)
    return st


class tt_stream_config(Structure):
    _fields_ = [
        ("n_slice_modes", c_int32),
        ("mode_sizes", POINTER(c_int64)),
        ("ranks", POINTER(c_int64)),
        ("compute", c_int),
        ("seed", c_uint64),
        ("init_cores", POINTER(c_double)),
        ("allocator", POINTER(tt_allocator)),
        ("hip_stream", c_void_p),
        ("keep_history", c_int32),
        ("history_capacity", c_int64),
        ("split_point", c_int32),
        ("flags", c_uint32),
    ]


_lib = None


class tt_server_config(Structure):
    _fields_ = [("max_wave", c_int32), ("lanes", c_int32), ("hbm_budget", c_uint64)]


def load_library(path: str = LIB_PATH):
    """Load libttstream.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    sv = c_void_p
    proto = {
        "tt_stream_create": (c_int, [POINTER(tt_stream_config), POINTER(c_void_p)]),
        "tt_stream_push_slice": (c_int, [sv, sv, c_int, c_int]),
        "tt_stream_reconstruct": (c_int, [sv, sv, c_int, c_int]),
        "tt_stream_destroy": (c_int, [sv]),
        "tt_stream_synchronize": (c_int, [sv]),
        "tt_stream_wait_update": (c_int, [sv]),
        "tt_stream_time": (c_int, [sv, POINTER(c_int64)]),
        "tt_stream_info": (c_int, [sv, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32), POINTER(c_int64)]),
        "tt_stream_get_state": (c_int, [sv, POINTER(c_double), POINTER(c_double), POINTER(c_int64)]),
        "tt_stream_set_state": (c_int, [sv, POINTER(c_double), POINTER(c_double), c_int64]),
        "tt_stream_get_history": (c_int, [sv, POINTER(c_double), c_int64, POINTER(c_int64)]),
        "tt_clamp_ranks": (c_int, [c_int32, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)]),
        "tt_stream_last_push_ms": (c_int, [sv, POINTER(c_float)]),
        "tt_stream_op_profile": (c_int, [sv, c_int64, POINTER(c_int32), POINTER(c_int64), POINTER(c_double),
                                         POINTER(c_int64)]),
        "tt_stream_pass_profile": (c_int, [sv, POINTER(c_float)]),
        "tt_stream_pass_kernels": (c_int, [sv, POINTER(c_int32), POINTER(c_int32)]),
        "tt_stream_time_passes": (c_int, [sv, POINTER(c_void_p), c_int32, c_int, c_int32, POINTER(c_float)]),
        "tt_last_error_string": (c_char_p, []),
        "tt_version": (c_char_p, []),
        "tt_batch_create": (c_int, [POINTER(c_void_p), c_int32, sv, POINTER(c_void_p)]),
        "tt_batch_push": (c_int, [sv, POINTER(c_void_p), c_int]),
        "tt_batch_synchronize": (c_int, [sv, POINTER(c_int32)]),
        "tt_batch_info": (c_int, [sv, POINTER(c_int32), POINTER(c_int32)]),
        "tt_batch_use_graph": (c_int, [sv, c_int32]),
        "tt_server_create": (c_int, [POINTER(tt_server_config), POINTER(c_void_p)]),
        "tt_server_add": (c_int, [sv, sv, POINTER(c_int32)]),
        "tt_server_submit": (c_int, [sv, c_int32, sv, c_int, c_uint64]),
        "tt_server_poll": (c_int, [sv, POINTER(c_int32)]),
        "tt_server_drain": (c_int, [sv]),
        "tt_server_take": (c_int, [sv, c_int64, POINTER(c_uint64), POINTER(c_double), POINTER(c_int32),
                                   POINTER(c_int64)]),
        "tt_server_stats": (c_int, [sv, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64), POINTER(c_int64),
                                    POINTER(c_uint64)]),
        "tt_server_destroy": (c_int, [sv]),
        "tt_batch_destroy": (c_int, [sv]),
        "tt_kernel_pass1": (c_int, [sv, c_int, c_int64, c_int64, c_int32, sv, sv, sv, sv, sv]),
        "tt_kernel_pass1_workspace": (c_size_t, [c_int64, c_int64, c_int32]),
        "tt_kernel_pass1_noalloc": (c_int, [sv, c_int, c_int64, c_int64, c_int32, sv, sv, sv, sv]),
        "tt_kernel_pass1_noalloc_max": (c_size_t, []),
        "tt_kernel_pass2": (c_int, [sv, c_int, c_int64, c_int64, c_int32, sv, sv, sv, sv]),
        "tt_kernel_qr": (c_int, [c_int32, c_int32, sv, sv, sv, sv, sv]),
        "tt_kernel_pass1_bf16": (c_int, [sv, c_int, c_int64, c_int64, c_int32, sv, sv, sv, sv, sv]),
        "tt_kernel_pass1_bf16_workspace": (c_size_t, [c_int64, c_int64, c_int32]),
        "tt_kernel_pass2_bf16": (c_int, [sv, c_int, c_int64, c_int64, c_int32, sv, sv, sv, sv, sv]),
        "tt_kernel_pass2_bf16_workspace": (c_size_t, [c_int64, c_int64, c_int32]),
    }
    for name, (res, args) in proto.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != TT_OK:
        raise TTError(status, where, load_library().tt_last_error_string().decode())


def _i64(values: Sequence[int]):
    arr = (c_int64 * len(values))(*[int(v) for v in values])
    return arr


# ------------------------------------------------------------- C-named calls
def tt_clamp_ranks(modes: Sequence[int], ranks: Sequence[int]):
    lib = load_library()
    m = len(modes)
    out = (c_int64 * m)()
    _check(lib.tt_clamp_ranks(m, _i64(modes), _i64(ranks), out), "tt_clamp_ranks")
    return [int(v) for v in out]


def tt_stream_create(modes, ranks, *, init_cores: Optional[np.ndarray] = None, seed: int = 0,
                     hip_stream: int = 0, keep_history: bool = False, history_capacity: int = 0,
                     split_point: int = 0, flags: int = 0, compute: int = TT_F32,
                     allocator: Optional[tt_allocator] = None):
    lib = load_library()
    m = len(modes)
    cfg = tt_stream_config()
    cfg.n_slice_modes = m
    modes_a, ranks_a = _i64(modes), _i64(ranks)
    cfg.mode_sizes = ctypes.cast(modes_a, POINTER(c_int64))
    cfg.ranks = ctypes.cast(ranks_a, POINTER(c_int64))
    cfg.compute = compute
    cfg.seed = seed
    init = None
    if init_cores is not None:
        init = np.ascontiguousarray(init_cores, dtype=np.float64)
        cfg.init_cores = init.ctypes.data_as(POINTER(c_double))
    cfg.hip_stream = hip_stream or None
    cfg.keep_history = 1 if keep_history else 0
    cfg.history_capacity = history_capacity
    cfg.split_point = split_point
    cfg.flags = flags
    if allocator is not None:
        cfg.allocator = ctypes.pointer(allocator)
    h = c_void_p()
    _check(lib.tt_stream_create(byref(cfg), byref(h)), "tt_stream_create")
    return h


def tt_stream_push_slice(h, ptr: int, dtype: int, on_device: bool) -> int:
    return load_library().tt_stream_push_slice(h, c_void_p(ptr), dtype, 1 if on_device else 0)


def tt_stream_reconstruct(h, ptr: int, dtype: int, on_device: bool) -> int:
    return load_library().tt_stream_reconstruct(h, c_void_p(ptr), dtype, 1 if on_device else 0)


def tt_stream_destroy(h) -> int:
    return load_library().tt_stream_destroy(h)


def tt_stream_synchronize(h) -> int:
    return load_library().tt_stream_synchronize(h)


# ------------------------------------------------------------- wrapper
_TORCH_DT = {}


def _dtype_code_torch(t) -> int:
    import torch
    if not _TORCH_DT:
        _TORCH_DT.update({torch.float64: TT_F64, torch.float32: TT_F32, torch.bfloat16: TT_BF16})
    return _TORCH_DT[t.dtype]


def _dtype_code_np(a: np.ndarray) -> int:
    if a.dtype == np.float64:
        return TT_F64
    if a.dtype == np.float32:
        return TT_F32
    raise TypeError("host slices must be float64 or float32")


class TTStream:
    """One streaming TT decomposition on the current GPU.

    modes: slice mode sizes I_1..I_m; ranks: feasible TT-ranks r_1..r_m.
    init: optional (cores, g) in FP64 (cores[k] of shape (r_{k-1}, I_k, r_k)).
    stream: torch.cuda.Stream (default: the current stream).
    allocator: optional tt_allocator (make_allocator) for the handle's device
    memory; it must outlive the handle.
    sync_push, profile_ops, autotune, no_ortho, wave_plan: the TT_FLAG_*
    creation flags of tt_stream.h (wave_plan: plan the update for batched
    waves).
    """

    def __init__(self, modes, ranks, init=None, *, seed: int = 0, stream=None, keep_history: bool = False,
                 history_capacity: int = 0, split_point: int = 0, sync_push: bool = False,
                 profile_ops: bool = False, compute: str = "f32", autotune: bool = False,
                 no_ortho: bool = False, wave_plan: bool = False, allocator: Optional[tt_allocator] = None):
        self.modes = tuple(int(v) for v in modes)
        self.ranks = tuple(int(v) for v in ranks)
        self.n = int(np.prod(self.modes))
        flat = None
        if init is not None:
            cores, g = init
            parts = [np.asarray(c, dtype=np.float64).reshape(-1, order="F") for c in cores]
            parts.append(np.asarray(g, dtype=np.float64).reshape(-1))
            flat = np.concatenate(parts)
        self._stream = stream
        self._allocator = allocator
        sp = int(stream.cuda_stream) if stream is not None else self._current_stream_handle()
        self.hip_stream = sp
        self._h = tt_stream_create(self.modes, self.ranks, init_cores=flat, seed=seed, hip_stream=sp,
                                   keep_history=keep_history, history_capacity=history_capacity,
                                   split_point=split_point, compute={"f32": TT_F32, "bf16": TT_BF16}[compute],
                                   flags=(TT_FLAG_SYNC_PUSH if sync_push else 0)
                                   | (TT_FLAG_PROFILE_OPS if profile_ops else 0)
                                   | (TT_FLAG_AUTOTUNE if autotune else 0)
                                   | (TT_FLAG_NO_ORTHO if no_ortho else 0)
                                   | (TT_FLAG_WAVE_PLAN if wave_plan else 0),
                                   allocator=allocator)
        self._lib = load_library()

    @staticmethod
    def _current_stream_handle() -> int:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)

    # -- updates
    def push(self, x) -> None:
        """Push one slice: a torch CUDA tensor (any shape, numel = N, contiguous,
        memory with i_1 fastest) or a numpy array (shape `modes`, or flat
        with i_1 fastest)."""
        if isinstance(x, np.ndarray):
            flat = np.ascontiguousarray(x.reshape(-1, order="F") if x.ndim > 1 else x)
            if flat.size != self.n:
                raise ValueError("slice size mismatch")
            st = tt_stream_push_slice(self._h, flat.ctypes.data, _dtype_code_np(flat), False)
        else:
            if not x.is_cuda or not x.is_contiguous() or x.numel() != self.n:
                raise ValueError("device slice must be a contiguous CUDA tensor with N elements")
            st = tt_stream_push_slice(self._h, x.data_ptr(), _dtype_code_torch(x), True)
        _check(st, "tt_stream_push_slice")

    def push_ptr(self, ptr: int, dtype: int) -> int:
        """Push a device slice by raw pointer; returns the status code."""
        return tt_stream_push_slice(self._h, ptr, dtype, True)

    def synchronize(self) -> None:
        _check(tt_stream_synchronize(self._h), "tt_stream_synchronize")

    def wait_update(self) -> None:
        """Wait until the last pushed update has committed (the next update's
        preparation may still run)."""
        _check(self._lib.tt_stream_wait_update(self._h), "tt_stream_wait_update")

    def synchronize_status(self) -> int:
        return tt_stream_synchronize(self._h)

    def time(self) -> int:
        t = c_int64()
        _check(self._lib.tt_stream_time(self._h, byref(t)), "tt_stream_time")
        return int(t.value)

    def info(self):
        cl, rl, sp, db = c_int64(), c_int64(), c_int32(), c_int64()
        _check(self._lib.tt_stream_info(self._h, byref(cl), byref(rl), byref(sp), byref(db)), "tt_stream_info")
        return {"cores_len": cl.value, "r_last": rl.value, "split_point": sp.value, "device_bytes": db.value}

    # -- outputs
    def reconstruct(self, out=None, dtype: str = "float64"):
        """Reconstruction M_t of the latest slice.  With out=None returns a
        host numpy array of shape `modes`; with a CUDA tensor writes into it."""
        if out is None:
            arr = np.empty(self.n, dtype=np.float64 if dtype == "float64" else np.float32)
            code = TT_F64 if arr.dtype == np.float64 else TT_F32
            _check(tt_stream_reconstruct(self._h, arr.ctypes.data, code, False), "tt_stream_reconstruct")
            return arr.reshape(self.modes, order="F")
        _check(tt_stream_reconstruct(self._h, out.data_ptr(), _dtype_code_torch(out), True), "tt_stream_reconstruct")
        return out

    def get_state(self):
        info = self.info()
        cores = np.empty(info["cores_len"], dtype=np.float64)
        g = np.empty(info["r_last"], dtype=np.float64)
        t = c_int64()
        _check(self._lib.tt_stream_get_state(self._h, cores.ctypes.data_as(POINTER(c_double)),
                                             g.ctypes.data_as(POINTER(c_double)), byref(t)), "tt_stream_get_state")
        r = (1,) + self.ranks
        out, off = [], 0
        for k, n in enumerate(self.modes):
            sz = r[k] * n * r[k + 1]
            out.append(cores[off:off + sz].reshape((r[k], n, r[k + 1]), order="F"))
            off += sz
        return out, g, int(t.value)

    def set_state(self, cores, g, t: int = 0) -> None:
        flat = np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1, order="F") for c in cores])
        gg = np.ascontiguousarray(g, dtype=np.float64)
        _check(self._lib.tt_stream_set_state(self._h, flat.ctypes.data_as(POINTER(c_double)),
                                             gg.ctypes.data_as(POINTER(c_double)), int(t)), "tt_stream_set_state")

    def history(self, rows: int = 1 << 30) -> np.ndarray:
        rl = self.info()["r_last"]
        cap = min(rows, max(self.time(), 0))
        out = np.empty((max(cap, 1), rl), dtype=np.float64)
        got = c_int64()
        _check(self._lib.tt_stream_get_history(self._h, out.ctypes.data_as(POINTER(c_double)), cap, byref(got)),
               "tt_stream_get_history")
        return out[: got.value]

    def last_push_ms(self) -> float:
        v = c_float()
        _check(self._lib.tt_stream_last_push_ms(self._h, byref(v)), "tt_stream_last_push_ms")
        return float(v.value)

    def op_profile(self):
        """Per-operation device times (us) of the last push as a list of
        (kind, (m, n, k), us); needs flags including TT_FLAG_PROFILE_OPS."""
        cnt = c_int64()
        _check(self._lib.tt_stream_op_profile(self._h, 0, None, None, None, byref(cnt)), "tt_stream_op_profile")
        n = cnt.value
        kinds = (c_int32 * max(n, 1))()
        dims = (c_int64 * max(3 * n, 1))()
        us = (c_double * max(n, 1))()
        _check(self._lib.tt_stream_op_profile(self._h, n, kinds, dims, us, byref(cnt)), "tt_stream_op_profile")
        names = {1: "gemm", 2: "qr", 3: "normg", 4: "copy", 5: "commit"}
        return [(names.get(kinds[i], "?"), (dims[3 * i], dims[3 * i + 1], dims[3 * i + 2]), us[i]) for i in range(n)]

    def pass_profile(self):
        """Device ms of the last push's slice passes (needs profile_ops=True):
        dict with pass1_kernel, pass1, pass2_kernel, pass2 (the contraction
        kernel alone, and the whole pass with its reduction)."""
        ms = (c_float * 4)()
        _check(self._lib.tt_stream_pass_profile(self._h, ms), "tt_stream_pass_profile")
        return {"pass1_kernel": ms[0], "pass1": ms[1], "pass2_kernel": ms[2], "pass2": ms[3]}

    def pass_kernels(self):
        """Names of the contraction kernels of the two slice passes."""
        a, b = c_int32(), c_int32()
        _check(self._lib.tt_stream_pass_kernels(self._h, byref(a), byref(b)), "tt_stream_pass_kernels")
        return ("k_pass1", "k_pass1b")[a.value], ("k_pass2", "k_pass2b", "k_pass2s", "k_pass2g")[b.value]

    def time_passes(self, xs, reps: int = 50):
        """Average device us per launch of the slice-pass kernels, launched
        reps times back to back on the device slices xs (cycled): dict with
        pass1_kernel, pass1_reduce, pass2_kernel, pass2_reduce."""
        xs = list(xs)
        for x in xs:
            if not x.is_cuda or not x.is_contiguous() or x.numel() != self.n:
                raise ValueError("device slices must be contiguous CUDA tensors with N elements")
        ptrs = (c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        us = (c_float * 4)()
        _check(self._lib.tt_stream_time_passes(self._h, ptrs, len(xs), _dtype_code_torch(xs[0]), int(reps), us),
               "tt_stream_time_passes")
        return {"pass1_kernel": us[0], "pass1_reduce": us[1], "pass2_kernel": us[2], "pass2_reduce": us[3]}

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(tt_stream_destroy(self._h), "tt_stream_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- kernel calls
def tt_kernel_pass1(X, P: int, J: int, r: int, B, Z, workspace, flag, hip_stream: int = 0) -> int:
    return load_library().tt_kernel_pass1(c_void_p(X.data_ptr()), _dtype_code_torch(X), P, J, r,
                                          c_void_p(B.data_ptr()), c_void_p(Z.data_ptr()),
                                          c_void_p(workspace.data_ptr()), c_void_p(flag.data_ptr()),
                                          c_void_p(hip_stream or None))


def tt_kernel_pass1_noalloc(X, P: int, J: int, r: int, B, Z, flag, hip_stream: int = 0) -> int:
    return load_library().tt_kernel_pass1_noalloc(c_void_p(X.data_ptr()), _dtype_code_torch(X), P, J, r,
                                                  c_void_p(B.data_ptr()), c_void_p(Z.data_ptr()),
                                                  c_void_p(flag.data_ptr()), c_void_p(hip_stream or None))


def tt_kernel_pass1_noalloc_max() -> int:
    return int(load_library().tt_kernel_pass1_noalloc_max())


def tt_kernel_pass1_workspace(P: int, J: int, r: int) -> int:
    return int(load_library().tt_kernel_pass1_workspace(P, J, r))


def tt_kernel_pass2(X, P: int, J: int, r: int, A, Y, flag, hip_stream: int = 0) -> int:
    return load_library().tt_kernel_pass2(c_void_p(X.data_ptr()), _dtype_code_torch(X), P, J, r,
                                          c_void_p(A.data_ptr()), c_void_p(Y.data_ptr()),
                                          c_void_p(flag.data_ptr()), c_void_p(hip_stream or None))


def tt_kernel_pass1_bf16(X, P: int, J: int, r: int, B, Z, workspace, flag, hip_stream: int = 0) -> int:
    return load_library().tt_kernel_pass1_bf16(c_void_p(X.data_ptr()), _dtype_code_torch(X), P, J, r,
                                               c_void_p(B.data_ptr()), c_void_p(Z.data_ptr()),
                                               c_void_p(workspace.data_ptr()), c_void_p(flag.data_ptr()),
                                               c_void_p(hip_stream or None))


def tt_kernel_pass1_bf16_workspace(P: int, J: int, r: int) -> int:
    return int(load_library().tt_kernel_pass1_bf16_workspace(P, J, r))


def tt_kernel_pass2_bf16(X, P: int, J: int, r: int, A, Y, workspace, flag, hip_stream: int = 0) -> int:
    return load_library().tt_kernel_pass2_bf16(c_void_p(X.data_ptr()), _dtype_code_torch(X), P, J, r,
                                               c_void_p(A.data_ptr()), c_void_p(Y.data_ptr()),
                                               c_void_p(workspace.data_ptr()), c_void_p(flag.data_ptr()),
                                               c_void_p(hip_stream or None))


def tt_kernel_pass2_bf16_workspace(P: int, J: int, r: int) -> int:
    return int(load_library().tt_kernel_pass2_bf16_workspace(P, J, r))


def tt_kernel_qr(M, Q, R, workspace, hip_stream: int = 0) -> int:
    m, n = M.shape[1], M.shape[0]   # M given as a (n, m) C-contiguous tensor = m x n column-major
    return load_library().tt_kernel_qr(m, n, c_void_p(M.data_ptr()), c_void_p(Q.data_ptr()),
                                       c_void_p(R.data_ptr()) if R is not None else None,
                                       c_void_p(workspace.data_ptr()), c_void_p(hip_stream or None))


class TTBatch:
    """Streams advanced together (include/tt_batch.h): each push runs one
    update of every member with launches shared by all members, whatever their
    shapes.  Members must share the HIP stream they were created with and must
    outlive the batch.  graph=True replays pushes from captured HIP graphs
    (the members' stream must not be the default stream)."""

    def __init__(self, streams, graph: bool = False):
        self._lib = load_library()
        self.streams = list(streams)
        n = len(self.streams)
        handles = (c_void_p * n)(*[s._h.value for s in self.streams])
        sp = self.streams[0].hip_stream
        self._h = c_void_p()
        _check(self._lib.tt_batch_create(handles, n, c_void_p(sp or None), byref(self._h)), "tt_batch_create")
        if graph:
            _check(self._lib.tt_batch_use_graph(self._h, 1), "tt_batch_use_graph")

    def push(self, slices) -> None:
        """slices: one contiguous CUDA tensor per member, all of one dtype."""
        if len(slices) != len(self.streams):
            raise ValueError("one slice per member")
        for x, s in zip(slices, self.streams):
            if not x.is_cuda or not x.is_contiguous() or x.numel() != s.n:
                raise ValueError("device slices must be contiguous CUDA tensors with N elements")
        ptrs = (c_void_p * len(slices))(*[x.data_ptr() for x in slices])
        _check(self._lib.tt_batch_push(self._h, ptrs, _dtype_code_torch(slices[0])), "tt_batch_push")

    def synchronize(self):
        """Waits; returns the per-member counts of rejected (non-finite) slices."""
        rej = (c_int32 * len(self.streams))()
        st = self._lib.tt_batch_synchronize(self._h, rej)
        if st not in (TT_OK, TT_ERR_NONFINITE):
            _check(st, "tt_batch_synchronize")
        return [int(v) for v in rej]

    def info(self):
        n, g = c_int32(), c_int32()
        _check(self._lib.tt_batch_info(self._h, byref(n), byref(g)), "tt_batch_info")
        return {"streams": n.value, "groups": g.value}

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(self._lib.tt_batch_destroy(self._h), "tt_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TTServer:
    """Continuous-batching server over registered streams (include/tt_server.h).

    Requests are submitted as they arrive; poll() retires finished waves,
    admits queued requests (per-stream order, wave size, HBM budget) and
    launches the next wave on a free lane.  Registered streams must not be
    pushed directly."""

    def __init__(self, max_wave: int = 32, lanes: int = 2, hbm_budget: int = 0):
        self._lib = load_library()
        cfg = tt_server_config(max_wave, lanes, hbm_budget)
        self._h = c_void_p()
        _check(self._lib.tt_server_create(byref(cfg), byref(self._h)), "tt_server_create")
        self.streams = []

    def add(self, stream) -> int:
        i = c_int32()
        _check(self._lib.tt_server_add(self._h, stream._h, byref(i)), "tt_server_add")
        self.streams.append(stream)
        return i.value

    def submit(self, sid: int, x, tag: int) -> None:
        if not x.is_cuda or not x.is_contiguous() or x.numel() != self.streams[sid].n:
            raise ValueError("device slices must be contiguous CUDA tensors with N elements")
        _check(self._lib.tt_server_submit(self._h, sid, c_void_p(x.data_ptr()), _dtype_code_torch(x), tag),
               "tt_server_submit")

    def poll(self) -> int:
        d = c_int32()
        _check(self._lib.tt_server_poll(self._h, byref(d)), "tt_server_poll")
        return d.value

    def drain(self) -> None:
        _check(self._lib.tt_server_drain(self._h), "tt_server_drain")

    def take(self, cap: int = 1 << 16):
        """[(tag, latency_s, rejected)] of the requests retired since the last call."""
        tags = (c_uint64 * cap)()
        lat = (c_double * cap)()
        rej = (c_int32 * cap)()
        n = c_int64()
        _check(self._lib.tt_server_take(self._h, cap, tags, lat, rej, byref(n)), "tt_server_take")
        return [(int(tags[i]), float(lat[i]), int(rej[i])) for i in range(n.value)]

    def stats(self):
        w, r, q, f = c_int64(), c_int64(), c_int64(), c_int64()
        pb = c_uint64()
        _check(self._lib.tt_server_stats(self._h, byref(w), byref(r), byref(q), byref(f), byref(pb)),
               "tt_server_stats")
        return {"waves": w.value, "retired": r.value, "queued": q.value, "in_flight": f.value,
                "peak_bytes": pb.value}

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(self._lib.tt_server_destroy(self._h), "tt_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
