/*
 * tt_server.h - serving many streams on one GPU with continuous batching.
 *
 * A server owns the updates of the streams registered with it.  Requests (one
 * slice for one stream) are submitted as they arrive; each call of
 * tt_server_poll retires the waves that have finished, admits queued requests
 * into the next wave and launches it on a free lane (a HIP stream of the
 * server's), so requests that arrive while other waves run on the GPU join as
 * soon as a lane and memory allow, and waves on different lanes overlap on
 * the device.  A wave is one batched update of its members (include/
 * tt_batch.h), so every request computes bitwise what the same update
 * computes alone.
 *
 * Admission, in arrival order: a request is admitted when its stream has no
 * update in flight and no earlier request still queued (a stream's slices are
 * applied in order), the wave has fewer than max_wave members, all of the
 * wave's slices share one element type, and the device bytes of the admitted
 * and unfinished slices stay within hbm_budget (a request larger than the
 * whole budget is admitted alone).
 *
 * Slices are device pointers owned by the caller; a slice must stay valid
 * until its request is reported by tt_server_take.
 *
 * Registered streams.  While registered (from tt_server_add until the server
 * is destroyed), a stream's updates run on the server's lanes:
 * tt_stream_push_slice and tt_stream_time_passes on it return TT_ERR_STATE,
 * and tt_batch_create refuses it.  Every other tt_stream_* call that reads or
 * writes its state (synchronize, time, get_state, set_state, get_history,
 * reconstruct, op_profile, destroy) first waits for the last wave a lane
 * launched for it, so it sees the state after the stream's latest admitted
 * request.  Destroying a registered stream drops its still-queued requests
 * (they are never reported) and later submits for its id return
 * TT_ERR_INVALID_ARG.  A server handle is not internally synchronised.
 */
#ifndef TT_SERVER_H
#define TT_SERVER_H

#include "tt_stream.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tt_server tt_server;

typedef struct {
  int32_t max_wave;   /* most requests per wave, 1 .. 65535               */
  int32_t lanes;      /* waves in flight at once, 1 .. 8                  */
  uint64_t hbm_budget; /* bytes of admitted, unfinished slices; 0 = none   */
} tt_server_config;

/* Errors: INVALID_ARG (null or out-of-range fields), DEVICE, OOM. */
tt_status tt_server_create(const tt_server_config* cfg, tt_server** out);

/* Registers stream s (on the current device, not profiled, not registered
 * with any server) and returns its id (0, 1, ... in order of registration).
 * Errors: INVALID_ARG (null, destroyed or profiled stream, another device,
 * already registered here), STATE (registered with another server), DEVICE. */
tt_status tt_server_add(tt_server* sv, tt_stream* s, int32_t* id);

/* Queues one slice for stream id; tag is returned with the result.  The
 * request's latency is counted from this call.  Errors: INVALID_ARG (null
 * slice, bad dtype, unknown id or a destroyed stream). */
tt_status tt_server_submit(tt_server* sv, int32_t id, const void* slice, tt_dtype dtype, uint64_t tag);

/* Retires finished waves, admits queued requests and launches waves on free
 * lanes; never waits for the device.  *done (optional) receives the number of
 * requests retired by this call. */
tt_status tt_server_poll(tt_server* sv, int32_t* done);

/* Polls until no request is queued or in flight. */
tt_status tt_server_drain(tt_server* sv);

/* Moves up to cap retired requests, oldest first, into tags[], latency_s[]
 * (seconds from submit to the poll that saw the wave finish) and rejected[]
 * (1 if the slice was not finite and the stream's update was discarded);
 * *n receives the number moved. */
tt_status tt_server_take(tt_server* sv, int64_t cap, uint64_t* tags, double* latency_s, int32_t* rejected,
                         int64_t* n);

/* Counters: waves launched, requests retired, requests queued now, requests
 * in flight now, and the largest number of slice bytes admitted at once. */
tt_status tt_server_stats(const tt_server* sv, int64_t* waves, int64_t* retired, int64_t* queued,
                          int64_t* in_flight, uint64_t* peak_bytes);

/* Waits for the server's work and releases it; its streams stay valid and are
 * no longer registered (they may be pushed directly again). */
tt_status tt_server_destroy(tt_server* sv);

#ifdef __cplusplus
}
#endif

#endif /* TT_SERVER_H */
