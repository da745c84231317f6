"""MI355X (gfx950) Online TT-ALS: per-slice streaming Tensor-Train updates.

The product is the HIP shared library lib/libttstream.so with the C ABI in
include/tt_stream.h (batches of streams in include/tt_batch.h, serving in
include/tt_server.h, the kernel entry points in include/tt_kernels.h);
this package only builds it (build.py) and binds it (binding.py).
"""

from .binding import (  # noqa: F401
    TTStream,
    TTBatch,
    TTServer,
    TTError,
    load_library,
    tt_clamp_ranks,
    tt_stream_create,
    tt_stream_push_slice,
    tt_stream_reconstruct,
    tt_stream_destroy,
    tt_stream_synchronize,
    TT_F64,
    TT_F32,
    TT_BF16,
    LIB_PATH,
)
