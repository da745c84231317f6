"""Reconstruction error (oracle; test infrastructure only).

Section 5.1 defines RE as the Frobenius norm of the difference between the
original and the reconstructed tensor over the norm of the original.  For a
stream reconstructed slice by slice, the squared norms add over slices.
"""

from __future__ import annotations

import numpy as np


def relative_error(X: np.ndarray, Xhat: np.ndarray) -> float:
    X = np.asarray(X, dtype=np.float64)
    d = X - np.asarray(Xhat, dtype=np.float64)
    return float(np.sqrt(np.sum(d * d) / np.sum(X * X)))


def stream_re(errors, norms) -> float:
    """RE over a stream from per-slice ||X_t - M_t|| and ||X_t||."""
    e = np.asarray(errors, dtype=np.float64)
    n = np.asarray(norms, dtype=np.float64)
    return float(np.sqrt(np.sum(e * e) / np.sum(n * n)))
