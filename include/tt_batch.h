/*
 * tt_batch.h - many streams advanced together on one GPU.
 *
 * Each stream's update (Algorithm 1) is a fixed sequence of steps: chain
 * steps run by one workgroup, whole-GPU products, and the two slice passes.
 * Streams created with the same mode sizes, TT-ranks and split point have
 * identical step sequences; a batch groups such streams and launches every
 * step once for the whole group (the chain steps with one workgroup per
 * stream, the other kernels with a stream index in the grid).  Every stream
 * is computed exactly as when pushed alone (same kernels, same arithmetic,
 * same order), so its results are bitwise the same.  Streams of different
 * shapes form separate groups, launched one after the other on the batch's
 * HIP stream.
 *
 * All streams must live on the current device, were created with the
 * batch's hip_stream, and must outlive the batch.  Calls are stream-ordered
 * like tt_stream_push_slice; a handle is not internally synchronised.
 */
#ifndef TT_BATCH_H
#define TT_BATCH_H

#include "tt_stream.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tt_batch tt_batch;

/* Groups n >= 1 distinct streams.  Errors: INVALID_ARG (null, n < 1,
 * duplicates, a stream created on another HIP stream or device, a stream
 * created with TT_FLAG_PROFILE_OPS), OOM, DEVICE. */
tt_status tt_batch_create(tt_stream* const* streams, int32_t n, void* hip_stream, tt_batch** out);

/* One update of every member: slices[i] is member i's next slice, a device
 * pointer of `dtype` elements laid out as in tt_stream_push_slice.  A
 * non-finite slice is rejected for its own stream only (reported by
 * tt_batch_synchronize).  Errors: INVALID_ARG, DEVICE. */
tt_status tt_batch_push(tt_batch* b, const void* const* slices, tt_dtype dtype);

/* Waits for the batch's work.  rejected (optional, n entries) receives for
 * each member the number of slices rejected since the previous call.
 * Returns TT_ERR_NONFINITE if any member rejected a slice, else TT_OK. */
tt_status tt_batch_synchronize(tt_batch* b, int32_t* rejected);

/* Number of members and of shape groups. */
tt_status tt_batch_info(const tt_batch* b, int32_t* n_streams, int32_t* n_groups);

tt_status tt_batch_destroy(tt_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* TT_BATCH_H */
