"""Pins of the stream reconstruction error (Section 5.1's RE) that every RE
gate uses, on the oracle and on the GPU side.

Section 5.1 defines RE as ||X - X^||_F / ||X||_F of the whole tensor.  For a
stream reconstructed slice by slice (the output sequence of Algorithm 1: slice
t is reconstructed from the time-t decomposition) the whole tensor is the
slices stacked along the temporal mode, so RE must equal the Frobenius ratio
of the stacked tensors, not a mean of per-slice ratios.
"""

import numpy as np

from oracle import metrics, ttals
from ttgen import config_c1, exact_tt_stream


def test_stream_re_worked_example():
    # errors (1, 0) against norms (1, 10): the stacked ratio is sqrt(1 / 101);
    # the mean of the per-slice ratios would be 0.5
    assert abs(metrics.stream_re([1.0, 0.0], [1.0, 10.0]) - np.sqrt(1.0 / 101.0)) <= 1e-16
    # a single slice reduces to its own ratio
    assert metrics.stream_re([3.0], [4.0]) == 0.75


def test_relative_error_worked_example():
    X = np.array([[3.0, 0.0], [0.0, 4.0]])
    Xh = np.array([[3.0, 0.0], [0.0, 0.0]])
    assert metrics.relative_error(X, Xh) == 0.8          # ||(0,0,0,4)|| / ||(3,0,0,4)||
    assert metrics.relative_error(X, X) == 0.0


def _stacked(slices, Ms):
    X = np.stack([np.asarray(x, dtype=np.float64) for x in slices], axis=-1)
    Xh = np.stack([np.asarray(m, dtype=np.float64) for m in Ms], axis=-1)
    return X, Xh


def test_stream_re_equals_re_of_the_stacked_stream():
    """StreamResult.re and metrics.stream_re both equal relative_error of the
    stacked slices and their reconstructions, on a stream whose slices differ
    in norm (so a mean of ratios differs from the stacked ratio)."""
    st = config_c1(T=30)
    cores, g = st.init()
    slices = [x * (1.0 + 4.0 * (t % 3)) for t, x in enumerate(st.frames(1, st.T))]
    res = ttals.run_stream(slices, cores, g, keep_M=True)
    X, Xh = _stacked(slices, [i.M for i in res.infos])
    ref = metrics.relative_error(X, Xh)
    assert abs(res.re - ref) <= 1e-13 * ref
    assert abs(metrics.stream_re(res.E, res.Xnorm) - ref) <= 1e-13 * ref
    mean_of_ratios = float(np.mean(res.E / res.Xnorm))
    assert abs(mean_of_ratios - ref) > 1e-3 * ref   # the example separates the two readings


def test_stream_re_on_a_higher_order_stream():
    st = exact_tt_stream((6, 5, 4), (3, 3, 2), (3, 3, 2), 12, 71, 72, sigma=5e-2)
    cores, g = st.init()
    slices = list(st.frames(1, st.T))
    res = ttals.run_stream(slices, cores, g, keep_M=True)
    X, Xh = _stacked(slices, [i.M for i in res.infos])
    assert abs(res.re - metrics.relative_error(X, Xh)) <= 1e-13 * res.re
    # the per-slice errors are ||X_t - M_t|| of the stacked slices
    for t, info in enumerate(res.infos):
        assert abs(info.E - np.linalg.norm(X[..., t] - Xh[..., t])) <= 1e-12 * info.Xnorm
