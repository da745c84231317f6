"""Seeded synthetic inputs for Online TT-ALS streams.

This package only draws random numbers and builds synthetic slice streams and
random initial cores.  It holds none of the Online TT-ALS update arithmetic, so
both the FP64 oracle tests and the GPU path's tests can take their inputs from
it without sharing any of the method's code.

Conventions: every tensor is dense with the first index fastest (the
column-major matricisation of Section 2.1).  A slice of an order-(m+1) stream is
an array of shape (I_1, ..., I_m); a core is (r_{k-1}, I_k, r_k).
"""

from .streams import (  # noqa: F401
    StreamSpec,
    config_c1,
    config_c2,
    config_c3,
    config_c4_specs,
    config_c4_streams,
    init_cores,
    flatten_cores,
    exact_tt_stream,
    tt_full,
    slice_f_order,
)
