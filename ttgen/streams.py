"""Seeded synthetic slice streams and initial cores (inputs only).

Every stream here is a low-TT-rank tensor whose last (temporal) bond is
contracted with a slowly varying vector h_t, plus i.i.d. Gaussian noise.  This
mirrors the workloads of Section 5.1: synthetic tensors built by contracting
random TT cores (with decaying spectra for the high-order case) and video-like
frame streams.  The paper's CDnet2014 videos are not available, so the
video-like streams stand in for them.

All randomness comes from numpy's PCG64 generator seeded explicitly.  Nothing
in this file performs any step of the Online TT-ALS update.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Iterator, List, Sequence, Tuple

import numpy as np


def slice_f_order(x: np.ndarray) -> np.ndarray:
    """Flat view of a slice with the first index fastest (vec of Section 2.1)."""
    return np.asarray(x).reshape(-1, order="F")


def tt_full(cores: Sequence[np.ndarray], h: np.ndarray | None = None) -> np.ndarray:
    """Dense tensor of a TT whose last bond is closed by vector h (or size 1).

    cores[k] has shape (r_{k-1}, I_k, r_k) with r_0 = 1.  Used by the
    generators to synthesise slices; the result has shape (I_1, ..., I_m).
    """
    modes = [c.shape[1] for c in cores]
    cores = list(cores)
    if h is not None:  # close the last bond first: the last core becomes (r, I_m, 1)
        c = cores[-1]
        cores[-1] = (c.reshape(-1, c.shape[2], order="F") @ np.asarray(h, dtype=np.float64)).reshape(
            c.shape[0], c.shape[1], 1, order="F")
    acc = np.ones((1, 1))  # (prod I so far) x r
    for c in cores:
        r0, n, r1 = c.shape
        # Fortran-ordered product, so the reshape below is a view, not a copy
        acc = np.asfortranarray(acc @ c.reshape(r0, n * r1, order="F")).reshape(-1, r1, order="F")
    assert acc.shape[1] == 1
    return acc[:, 0].reshape(modes, order="F")


def init_cores(modes: Sequence[int], ranks: Sequence[int], seed: int):
    """Random initial cores and temporal vector, i.i.d. N(0,1) in FP64.

    The paper initialises the cores randomly without naming a distribution
    (Section 3.4); i.i.d. standard normal entries are used.  ranks = (r_1..r_m),
    r_0 = 1 implicit; g has r_m entries.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    r = [1] + list(ranks)
    cores = [rng.standard_normal((r[k], modes[k], r[k + 1])) for k in range(len(modes))]
    g = rng.standard_normal(r[-1])
    return cores, g


def flatten_cores(cores: Sequence[np.ndarray], g: np.ndarray) -> np.ndarray:
    """Concatenate G_1..G_m then g, each with the first index fastest (FP64)."""
    parts = [np.asarray(c, dtype=np.float64).reshape(-1, order="F") for c in cores]
    parts.append(np.asarray(g, dtype=np.float64).reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


@dataclass
class StreamSpec:
    """A synthetic stream: slice modes, model TT-ranks, length and generator."""

    name: str
    modes: Tuple[int, ...]
    ranks: Tuple[int, ...]          # model ranks r_1..r_m (already feasible)
    T: int
    dtype: type
    data_seed: int
    init_seed: int
    _frame_fn: object = field(repr=False, default=None)

    @property
    def n_elems(self) -> int:
        return int(np.prod(self.modes))

    def frame(self, t: int) -> np.ndarray:
        """Slice X_t (t = 1..T) as an F-ordered array of shape modes."""
        return self._frame_fn(t)

    def frames(self, t0: int, t1: int) -> Iterator[np.ndarray]:
        for t in range(t0, t1 + 1):
            yield self.frame(t)

    def init(self):
        return init_cores(self.modes, self.ranks, self.init_seed)


def _walk(rng, h0, T, step):
    hs = [h0]
    for _ in range(T):
        hs.append(hs[-1] + step * rng.standard_normal(h0.shape))
    return hs


def _tt_sq_norm(cores, h) -> float:
    """||TT(cores) x_last h||_F^2 by the left-to-right Gram recursion."""
    W = np.ones((1, 1))
    for c in cores:
        r0, n, r1 = c.shape
        W = sum(c[:, i, :].T @ W @ c[:, i, :] for i in range(n))
    h = np.asarray(h, dtype=np.float64)
    return float(h @ W @ h)


def exact_tt_stream(modes, true_ranks, model_ranks, T, data_seed, init_seed,
                    sigma=0.0, walk_step=0.05, dtype=np.float64, decay=None,
                    name="exact_tt", noise_rel=None):
    """Exact TT-rank stream: X_t = TT(C_1..C_m) x_last h_t + sigma * noise.

    C_k are i.i.d. N(0,1) of shape (q_{k-1}, I_k, q_k) with q = true_ranks;
    h_t is a Gaussian random walk of dimension q_m.  With decay=c the b-th
    output slice of every core is scaled by c**b (decaying spectra).
    """
    rng = np.random.Generator(np.random.PCG64(data_seed))
    q = [1] + list(true_ranks)
    cores = []
    for k in range(len(modes)):
        c = rng.standard_normal((q[k], modes[k], q[k + 1]))
        if decay is not None:
            c *= (decay ** np.arange(q[k + 1]))[None, None, :]
        cores.append(c)
    hs = _walk(rng, rng.standard_normal(q[-1]), T, walk_step)
    noise_seed = int(rng.integers(0, 2**62))
    if noise_rel is not None:  # noise_rel times the RMS of the first slice's signal
        sigma = noise_rel * np.sqrt(_tt_sq_norm(cores, hs[1]) / float(np.prod(modes)))

    def frame(t):
        x = tt_full(cores, hs[t])
        if sigma > 0.0:
            nr = np.random.Generator(np.random.PCG64([noise_seed, t]))
            x = x + sigma * nr.standard_normal(x.shape)
        return np.asfortranarray(x.astype(dtype))

    return StreamSpec(name, tuple(modes), tuple(model_ranks), T, dtype,
                      data_seed, init_seed, frame)


def config_c1(sigma: float = 1e-3, T: int = 200, model_ranks=(4, 4)) -> StreamSpec:
    """Order-3 stream of 32x32 FP64 slices, exact TT-rank 4 plus N(0, sigma^2).

    True cores C_1 (1x32x4), C_2 (4x32x4) i.i.d. N(0,1); h_0 ~ N(0, I_4),
    h_t = h_{t-1} + 0.05 xi_t.
    """
    return exact_tt_stream((32, 32), (4, 4), model_ranks, T, 1001, 2001,
                           sigma=sigma, walk_step=0.05, dtype=np.float64,
                           name="c1_order3_32x32_r4")


def config_c2(T: int = 1000) -> StreamSpec:
    """Order-4 video-like stream: 240x320x3 FP32 frames in about [0, 1].

    Non-negative base cores U[0,1): C_1 1x240x16, C_2 16x320x16, C_3 16x3x16.
    Each core drifts smoothly, C_k(t) = C_k(0) * (1 + 0.1 sin(2 pi t/T_k + phi)),
    with a period T_k ~ U[200, 1000] per core and an elementwise phase phi.
    h_t is a positive smooth walk.  Frame 0's signal is scaled to max 1 and
    N(0, 1e-2^2) noise is added (not clipped, so the low rank is kept).
    """
    modes, q = (240, 320, 3), (16, 16, 16)
    rng = np.random.Generator(np.random.PCG64(1002))
    rr = [1] + list(q)
    base = [rng.uniform(0.0, 1.0, (rr[k], modes[k], rr[k + 1])) for k in range(3)]
    periods = rng.uniform(200.0, 1000.0, 3)
    phases = [rng.uniform(0.0, 2 * np.pi, b.shape) for b in base]
    h0 = rng.uniform(0.5, 1.5, q[-1])
    steps = rng.standard_normal((T + 1, q[-1]))
    noise_seed = int(rng.integers(0, 2**62))

    def h_at(t):
        h = h0.copy()
        for s in range(1, t + 1):
            h = np.abs(h + 0.02 * steps[s])
        return h

    def signal(t):
        cores = [b * (1.0 + 0.1 * np.sin(2 * np.pi * t / periods[k] + phases[k]))
                 for k, b in enumerate(base)]
        return tt_full(cores, h_at(t))

    scale = 1.0 / float(np.max(signal(0)))

    def frame(t):
        nr = np.random.Generator(np.random.PCG64([noise_seed, t]))
        x = scale * signal(t) + 1e-2 * nr.standard_normal(modes)
        return np.asfortranarray(x.astype(np.float32))

    return StreamSpec("c2_video_240x320x3_r16", modes, (16, 16, 16), T, np.float32,
                      1002, 2002, frame)


C3_MODES = (8, 9, 15, 8, 16, 15, 3, 1, 1)
C3_RANKS = (8, 32, 32, 32, 32, 32, 32, 32, 32)


def config_c3(T: int = 500) -> StreamSpec:
    """High-order stream: 1080x1920x3 FP32 frames as the order-9 slice
    (8,9,15,8,16,15,3,1,1), 6,220,800 entries, TT-rank 32 clamped to
    (8,32,...,32).

    True cores are i.i.d. N(0,1) with output slice b scaled by 0.85**b
    (decaying spectra, as the synthetic tensors of Section 5.1), h_t a
    Gaussian random walk (step 0.05), signal scaled to unit rms at t=0, and
    noise of standard deviation 1e-2 times that rms.
    """
    modes, q = C3_MODES, C3_RANKS
    rng = np.random.Generator(np.random.PCG64(1003))
    rr = [1] + list(q)
    cores = []
    for k in range(len(modes)):
        c = rng.standard_normal((rr[k], modes[k], rr[k + 1]))
        c *= (0.85 ** np.arange(rr[k + 1]))[None, None, :]
        cores.append(c)
    hs = _walk(rng, rng.standard_normal(q[-1]), T, 0.05)
    noise_seed = int(rng.integers(0, 2**62))
    # Left block (I_1 I_2 I_3) x r_3 and right block r_3 x (I_4..I_9) x r_9.
    left = tt_full_left(cores[:3])                      # 1080 x 32
    right = tt_full_middle(cores[3:])                   # (32*5760) x 32
    P = int(np.prod(modes[:3]))
    J = int(np.prod(modes[3:]))

    def signal(t):
        rt = (right @ hs[t]).reshape(q[2], J, order="F")
        return left @ rt                                # P x J

    s0 = signal(0)
    scale = 1.0 / float(np.sqrt(np.mean(s0 * s0)))

    def frame(t):
        nr = np.random.Generator(np.random.PCG64([noise_seed, t]))
        x = scale * signal(t) + 1e-2 * nr.standard_normal((P, J))
        return np.asfortranarray(x.astype(np.float32).reshape(modes, order="F"))

    return StreamSpec("c3_order9_1080x1920x3_r32", modes, q, T, np.float32,
                      1003, 2003, frame)


def tt_full_left(cores):
    """(I_1..I_k) x r_k matrix of the contraction of cores 1..k (r_0 = 1)."""
    acc = np.ones((1, 1))
    for c in cores:
        r0, n, r1 = c.shape
        acc = (acc @ c.reshape(r0, n * r1, order="F")).reshape(-1, r1, order="F")
    return acc


def tt_full_middle(cores):
    """(r_a * prod I) x r_b matrix of a chain of cores with open end bonds."""
    r_a = cores[0].shape[0]
    acc = np.eye(r_a).reshape(r_a, r_a)             # rows: (a, i...) ; cols: bond
    rows = r_a
    for c in cores:
        r0, n, r1 = c.shape
        acc = (acc @ c.reshape(r0, n * r1, order="F")).reshape(rows * n, r1, order="F")
        rows *= n
    return acc


def config_c4_specs(seed: int = 1004, n_streams: int = 64):
    """Shapes of the batched workload: orders 3-5, modes U{16..256},
    ranks in {4,8,16,32} (uniform per stream, then clamped by the caller)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs: List[dict] = []
    for s in range(n_streams):
        order = int(rng.integers(3, 6))
        modes = tuple(int(v) for v in rng.integers(16, 257, order - 1))
        rank = int(rng.choice([4, 8, 16, 32]))
        specs.append({"stream": s, "modes": modes, "rank": rank})
    return specs


def config_c4_streams(n_streams: int = 64, seed: int = 1004, T: int = 300, max_elems: int = 1 << 22,
                      clamp=None, noise_rel: float = 1e-2) -> List[StreamSpec]:
    """The batched workload: streams of order 3-5 (slices of order 2-4), each
    slice mode U{16..256}, one rank drawn from {4, 8, 16, 32} per stream and
    clamped to feasibility by `clamp(modes, ranks)`, low TT-rank plus Gaussian
    noise of noise_rel times the signal's RMS.  Shapes whose slice exceeds
    max_elems entries are drawn again, so a round of slices fits a bounded
    amount of device memory."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs: List[StreamSpec] = []
    while len(specs) < n_streams:
        order = int(rng.integers(3, 6))
        modes = tuple(int(v) for v in rng.integers(16, 257, order - 1))
        rank = int(rng.choice([4, 8, 16, 32]))
        if int(np.prod(modes)) > max_elems:
            continue
        ranks = tuple(int(v) for v in (clamp(modes, [rank] * len(modes)) if clamp else [rank] * len(modes)))
        q = len(specs)
        ds, is_ = seed * 1000 + 2 * q, seed * 1000 + 2 * q + 1
        specs.append(exact_tt_stream(modes, ranks, ranks, T, ds, is_, noise_rel=noise_rel,
                                     dtype=np.float32, name=f"c4_{q}_order{order}"))
    return specs
