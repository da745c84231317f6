/*
 * tt_batch.h - many streams advanced together on one GPU.
 *
 * Each stream's update (Algorithm 1's loop body) is a fixed sequence of
 * steps: chain steps run by one workgroup, whole-GPU products, and the two
 * slice passes (Eq. 5 evaluated at the split point, Section 4.2).  A batch
 * cuts every member's sequence at the two passes into three phases and runs
 * slot w of every member's phase in one launch (chain segment w with one
 * workgroup per member, then product w of the members that have one); each
 * pass runs as one launch per kernel template shape over the members of that
 * shape; the pass launches of fewer than 256 blocks run on a HIP stream the
 * batch creates for itself (default priority, non-blocking), forked from and
 * joined back to hip_stream by events within each push, so that they run
 * beside the wider ones.  Members may differ in order, mode sizes, ranks, split point and
 * contraction precision.  Every member is computed exactly as when pushed
 * alone (same kernels, launch shapes and arithmetic order), so its results
 * are bitwise the same.
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

/* Groups n >= 1 distinct streams; creates the batch's own side stream and
 * its two events (released by tt_batch_destroy).  Errors: INVALID_ARG (null,
 * n < 1, duplicates, a stream created on another HIP stream or device, a
 * stream created with TT_FLAG_PROFILE_OPS), OOM, DEVICE (also when the side
 * stream or its events cannot be created). */
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

/* Replays each push from a captured HIP graph (enable != 0): the first push
 * through each of the batch's eight descriptor slots captures the push's
 * descriptor upload and launches into a graph; later pushes rewrite the
 * slot's descriptors and launch the graph.  Results are bitwise those of the
 * eager path.  Needs a batch created on a non-default hip_stream
 * (TT_ERR_UNSUPPORTED otherwise).  Errors: INVALID_ARG, DEVICE. */
tt_status tt_batch_use_graph(tt_batch* b, int32_t enable);

/* Number of members and of distinct update structures among them. */
tt_status tt_batch_info(const tt_batch* b, int32_t* n_streams, int32_t* n_groups);

tt_status tt_batch_destroy(tt_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* TT_BATCH_H */
