/*
 * tt_stream.h - C ABI of the MI355X (gfx950) Online TT-ALS streaming library.
 *
 * The library maintains the Tensor-Train decomposition of a stream of
 * order-(n-1) slices X_t of size I_1 x ... x I_m (m = n - 1 slice modes) and,
 * for every slice pushed, performs one update of Online TT-ALS (Algorithm 1,
 * Section 3.4 of "Online TT-ALS for Streaming Tensor Decomposition with
 * Incremental Orthogonalization"):
 *   1. normalise the temporal vector g and right-orthogonalise the cores by an
 *      LQ sweep (Section 3.4.1);
 *   2. build the right interfaces B_k from the time t-1 cores;
 *   3. for k = 1..m solve the local least-squares problem in closed form
 *      (Eq. 5, G~_k = A_k^T x X_t x B_k^T), re-orthogonalise by thin QR and
 *      update the left interface A_{k+1} (Section 3.4.2);
 *   4. set the new temporal-core row g_n[t] = A_n^T vec(X_t).
 *
 * Conventions
 *   - Every dense array has its FIRST index fastest (the column-major
 *     matricisation of Section 2.1).  A slice is I_1*...*I_m contiguous
 *     elements with i_1 fastest.  A core G_k is r_{k-1} x I_k x r_k with the
 *     r_{k-1} index fastest.  A caller holding a C-order (row-major) tensor
 *     passes its modes in reverse order.
 *   - TT-ranks are given as r_1..r_m; r_0 = 1 is implicit and r_m is the bond
 *     between the last slice core and the temporal core.
 *   - Device pointers are HIP device pointers on the device that was current
 *     when the stream was created; host pointers are ordinary host memory.
 *   - All GPU work of a handle is ordered on the HIP stream given at creation
 *     (NULL = the legacy default stream).  Calls return before that work
 *     completes unless documented otherwise.
 *   - Ownership: the caller owns every buffer it passes (slices, outputs,
 *     initial cores) and the handle owns everything it allocates.  A device
 *     slice passed to tt_stream_push_slice must stay valid until the stream
 *     has been synchronised; the library never keeps the pointer.
 *   - Errors: every entry point returns a tt_status; nothing throws or aborts
 *     across the ABI.  tt_last_error_string() describes the last failure of
 *     the calling thread.
 *   - Threads: a handle is not internally synchronised (one host thread per
 *     handle at a time); distinct handles are independent.
 */
#ifndef TT_STREAM_H
#define TT_STREAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tt_stream tt_stream;  /* opaque, library-owned */

typedef enum {
  TT_OK = 0,
  TT_ERR_INVALID_ARG = 1,  /* null/destroyed handle, null pointer, bad enum  */
  TT_ERR_SHAPE = 2,        /* m < 1, a mode size or rank < 1, size overflow  */
  TT_ERR_RANK = 3,         /* infeasible TT-ranks (see tt_clamp_ranks)        */
  TT_ERR_OOM = 4,          /* device or host allocation failed                */
  TT_ERR_DEVICE = 5,       /* a HIP runtime call failed                       */
  TT_ERR_NONFINITE = 6,    /* a slice held NaN/Inf; that update was discarded */
  TT_ERR_STATE = 7,        /* call not valid in the current state             */
  TT_ERR_UNSUPPORTED = 8   /* combination not implemented                     */
} tt_status;

typedef enum { TT_F64 = 0, TT_F32 = 1, TT_BF16 = 2 } tt_dtype;

/* Optional device allocator.  alloc returns device memory of at least `bytes`
 * bytes (256-byte aligned) or NULL; free releases it.  NULL -> hipMalloc.
 * The handle calls alloc on the calling thread from tt_stream_create, and
 * lazily from tt_stream_push_slice (staging of host slices) and
 * tt_stream_reconstruct (reconstruction buffers); it calls free once for every
 * block it got, at tt_stream_destroy or when tt_stream_create fails.  A NULL
 * from alloc makes that call return OOM (create frees what it had). */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} tt_allocator;

/* Creation parameters (problem statement of Algorithm 1: data stream of
 * I_1 x ... x I_m slices and TT-ranks r). */
typedef struct {
  int32_t n_slice_modes;          /* m = n - 1 >= 1                                  */
  const int64_t* mode_sizes;      /* host array I_1..I_m, each >= 1                  */
  const int64_t* ranks;           /* host array r_1..r_m, feasible (tt_clamp_ranks)  */
  tt_dtype compute;               /* slice contractions: TT_F32 (default) or TT_BF16 */
  uint64_t seed;                  /* random N(0,1) initial cores if init_cores NULL  */
  const double* init_cores;       /* optional host FP64 G_1..G_m then g (r_m)        */
  const tt_allocator* allocator;  /* optional; NULL -> hipMalloc/hipFree             */
  void* hip_stream;               /* hipStream_t for all work; NULL = default stream */
  int32_t keep_history;           /* nonzero: keep the temporal rows g_n[1..t]       */
  int64_t history_capacity;       /* rows kept when keep_history (ring of that size) */
  int32_t split_point;            /* 0 = automatic; else k* in [1, m] (see below)    */
  uint32_t flags;                 /* TT_FLAG_* below                                  */
} tt_stream_config;

/* Flags. */
#define TT_FLAG_SYNC_PUSH 0x1u   /* push waits for its update and reports NONFINITE */
/* TT_FLAG_NO_ORTHO: the "w/o Ortho" ablation of Section 5, read as removing
 * the right-orthogonalisation of Section 3.4.1: g is not normalised and there
 * is no LQ sweep, so the right interfaces B_k built from the current cores are
 * not orthonormal.  Each local problem is then solved exactly with their Gram
 * matrix, G~_k = A_k^T X B_k^T (B_k B_k^T)^+ (the pseudo-inverse: (B_k B_k^T)^-1
 * when r_k <= J_k, else B_k (B_k^T B_k)^-2 B_k^T), with no shift, and the
 * forward sweep keeps its thin QR (G_k <- Fold(Q), A_{k+1} = A_k x G_k, g =
 * A_n^T vec(X)) exactly as without the flag.  In exact arithmetic this gives
 * the same M_t as the method (only the gauge of the right interfaces differs),
 * so the ablation can show the error growth of the Section 5 ablation table
 * only through the rounding that the Gram matrices' conditioning amplifies.
 * A non-positive Cholesky pivot of a Gram matrix rejects the update like a
 * non-finite slice.  TT-ranks <= 32, and r_k <= I_{k+1}..I_m below the split
 * point. */
#define TT_FLAG_NO_ORTHO 0x2u
#define TT_FLAG_PROFILE_OPS 0x4u /* time every chain operation (tt_stream_op_profile) */
/* TT_FLAG_AUTOTUNE: at create, time candidate launch shapes of the two slice
 * passes for this stream's shape and precision (with BF16, pass 2's kernel
 * too: staged through LDS or direct; once per process and shape, on
 * hip_stream, which is synchronised) and use the fastest; streams of one
 * shape then share the plan, alone or in a batch.  With split_point = 0 (and
 * without TT_FLAG_NO_ORTHO) it also picks k*: up to three split points whose
 * modelled side traffic (P_k + J_k) r_k is within 4x of the smallest are timed
 * with their tuned passes, and the fastest is used. */
#define TT_FLAG_AUTOTUNE 0x8u
/* TT_FLAG_WAVE_PLAN: plan the update for batched waves (tt_batch.h,
 * tt_server.h): FP64 products of up to 4e5 multiply-adds run inside the
 * one-workgroup chain segments rather than as whole-GPU launches of their own
 * (2e5 without the flag), and whole-GPU products of at least 4e6 compute
 * four outputs per thread.  In a wave every whole-GPU launch is another step
 * that all members wait for, and the members' large products run at once,
 * so the wave is faster; a stream alone is slower.  The
 * update is the same up to rounding either way, and a stream gives the same
 * bits alone or in a batch for a given flag. */
#define TT_FLAG_WAVE_PLAN 0x10u

/* Create a stream.  The initial cores are the paper's random initialisation
 * (Algorithm 1, first line): taken from init_cores, else i.i.d. N(0,1) from a
 * SplitMix64/Box-Muller generator seeded with `seed`.  The split point k*
 * chooses where the update's two passes over the slice meet: pass 1 forms
 * X^<k*> B_{k*}^T and pass 2 forms A_{k*+1}^T X^<k*> (both are Eq. 5 reassociated);
 * 0 picks the k* that minimises the passes' side traffic.
 * Errors: INVALID_ARG (null cfg/out), SHAPE, RANK, OOM, DEVICE, UNSUPPORTED. */
tt_status tt_stream_create(const tt_stream_config* cfg, tt_stream** out);

/* Push slice X_t (I_1*...*I_m elements, i_1 fastest) and run one update.
 * A stream registered with a server (include/tt_server.h) is updated through
 * the server only: pushing it directly returns STATE.
 * dtype is the slice's element type (F64, F32 or BF16; converted on load);
 * on_device != 0 means `slice` is a device pointer, else a host pointer (the
 * library copies it to the device first and the call returns after the copy).
 * A slice containing NaN/Inf leaves the state unchanged; that is reported by
 * the next tt_stream_synchronize (or by this call with TT_FLAG_SYNC_PUSH).
 * Errors: INVALID_ARG, STATE (registered with a server), OOM (host slice
 * staging), DEVICE, NONFINITE (sync mode only). */
tt_status tt_stream_push_slice(tt_stream* s, const void* slice, tt_dtype dtype, int on_device);

/* Write M_t = G_1 x ... x G_m x g_n[t], the reconstruction of the latest slice
 * from the time-t decomposition (Algorithm 1's output), into `out`
 * (I_1*...*I_m elements of `dtype`, F64 or F32).  Host outputs are complete
 * on return; device outputs are stream-ordered.
 * Errors: INVALID_ARG, STATE (no slice pushed yet), DEVICE. */
tt_status tt_stream_reconstruct(tt_stream* s, void* out, tt_dtype dtype, int on_device);

/* Destroy a handle and free everything it owns (waits for its work first; a
 * stream registered with a server leaves it, see include/tt_server.h).  The
 * library keeps a registry of live handles and checks every handle against
 * it before use, so any later call with the destroyed handle returns
 * INVALID_ARG. */
tt_status tt_stream_destroy(tt_stream* s);

/* Wait until the last pushed update has committed its result (Algorithm 1's
 * time-t output: the cores, g_n[t] and so M_t).  An update ends by preparing
 * the next one (the right-orthogonalisation of Section 3.4.1 and the right
 * interfaces, which read only the committed state); that work may still run
 * when this returns, and a following push waits for it on the handle's
 * stream.  This is the latency a slice sees when slices arrive with gaps.
 * It reports no rejected slice (tt_stream_synchronize does).  For a stream
 * registered with a server it waits for the stream's lane work.
 * Errors: INVALID_ARG, DEVICE. */
tt_status tt_stream_wait_update(tt_stream* s);

/* Wait for all work of the handle.  Returns NONFINITE if any update since the
 * previous call discarded a non-finite slice, else OK (or DEVICE). */
tt_status tt_stream_synchronize(tt_stream* s);

/* Number of committed updates t (waits for the handle's work). */
tt_status tt_stream_time(tt_stream* s, int64_t* t_out);

/* Sizes: total FP64 entries of G_1..G_m (cores_len), r_m, the split point
 * used, and the device bytes the handle holds.  Any output may be NULL. */
tt_status tt_stream_info(const tt_stream* s, int64_t* cores_len, int64_t* r_last,
                         int32_t* split_point, int64_t* device_bytes);

/* Copy the committed FP64 state to host memory: cores (cores_len entries,
 * G_1..G_m each first-index-fastest) and g (r_m entries).  Waits for the
 * handle's work.  Either output may be NULL. */
tt_status tt_stream_get_state(tt_stream* s, double* cores, double* g, int64_t* t_out);

/* Replace the state by host FP64 cores and g and set the update counter to t
 * (checkpoint/resume; injection of a reference state).  Waits first.  The
 * history (tt_stream_get_history) restarts empty at t. */
tt_status tt_stream_set_state(tt_stream* s, const double* cores, const double* g, int64_t t);

/* Copy up to `rows` of the kept temporal rows g_n[t] (Algorithm 1's output
 * per update), oldest first, to host memory (rows x r_m, row-major: one
 * r_m-vector per update).  The ring keeps the rows of the last
 * history_capacity updates since creation or the last set_state.  *rows_out
 * receives the number copied.  STATE if keep_history was 0. */
tt_status tt_stream_get_history(tt_stream* s, double* out, int64_t rows, int64_t* rows_out);

/* Largest feasible ranks <= ranks_in: r_k <= r_{k-1} I_k and r_{k-1} <= I_k r_k
 * (r_0 = 1), so every forward step is a thin QR of an (r_{k-1} I_k) x r_k
 * matrix and every sweep step a thin LQ of an r_{k-1} x (I_k r_k) matrix.
 * Errors: INVALID_ARG (null), SHAPE (m < 1 or sizes < 1). */
tt_status tt_clamp_ranks(int32_t m, const int64_t* modes, const int64_t* ranks_in, int64_t* ranks_out);

/* Device time of the last completed push in milliseconds, from the push to
 * the commit of its result (HIP events on the handle's stream; the
 * preparation of the next update that follows the commit is not included).
 * Waits for that update. */
tt_status tt_stream_last_push_ms(tt_stream* s, float* ms);

/* Per-operation device times of the last push, for a stream created with
 * TT_FLAG_PROFILE_OPS.  The update's small dense steps run as a list of
 * operations on one workgroup; each gets a start and end stamp from the
 * device wall clock.  For op i < min(count, cap): kinds[i] = 1 GEMM, 2 QR,
 * 3 g normalisation, 4 copy, 5 commit; dims[3i..3i+2] = (m, n, k) (GEMM:
 * rows, columns, depth; QR: rows, columns, reflector cap); us[i] = duration
 * in microseconds.  Operations launched over the whole GPU and the slice
 * passes are not listed (a kernel trace times them).  Waits for the handle's
 * work.  Errors: INVALID_ARG (null), STATE (flag not set or no push yet). */
tt_status tt_stream_op_profile(tt_stream* s, int64_t cap, int32_t* kinds, int64_t* dims, double* us,
                               int64_t* count);

/* Device times in milliseconds of the two slice passes of the last push, for
 * a stream created with TT_FLAG_PROFILE_OPS, from HIP events recorded on the
 * handle's stream: ms[0] pass 1's contraction kernel alone, ms[1] the whole
 * of pass 1 (with its partial-tile reduction), ms[2] and ms[3] the same for
 * pass 2 (equal when the pass is a single kernel).  ms: caller array of 4
 * floats.  Waits for the handle's work.  Errors: INVALID_ARG (null), STATE
 * (flag not set or no push yet). */
tt_status tt_stream_pass_profile(tt_stream* s, float* ms);

/* The contraction kernels the handle's slice passes launch (they follow its
 * precision and its launch plans, tuned or not): *pass1 = 0 for k_pass1 (FP32
 * MFMA) or 1 for k_pass1b (BF16 MFMA); *pass2 = 0 for k_pass2 (FP32 MFMA),
 * 1 for k_pass2b (BF16 MFMA, slice read straight into registers), 2 for
 * k_pass2s (BF16 MFMA, slice staged through LDS) or 3 for k_pass2g (FP32
 * MFMA, whole-slab loads in 16-row groups; FP32 slices with 4 <= P <= 1280
 * and r <= 32 at the split point (P J < 2^30 when P % 4 != 0), where slices
 * of the other dtypes use k_pass2).  Errors: INVALID_ARG (null). */
tt_status tt_stream_pass_kernels(const tt_stream* s, int32_t* pass1, int32_t* pass2);

/* Average device time per launch, in microseconds, of the handle's slice-pass
 * kernels (the contractions of Section 4.2 at the split point, with the
 * interfaces of the last update): each kernel is launched `reps` times back
 * to back on the handle's stream between two HIP events, after one untimed
 * launch, launch i reading slices[i % nslices] (several resident slices keep
 * the reads out of the caches).  us[0] pass 1's contraction kernel, us[1] its
 * partial-tile reduction, us[2] pass 2's contraction kernel, us[3] its
 * reduction (about 0 when the pass has none).  slices: nslices device
 * pointers, layout and dtype as for tt_stream_push_slice.  The passes'
 * outputs are per-update scratch and the state is not changed; waits for the
 * handle's work.  us: caller array of 4 floats.  Errors: INVALID_ARG (null,
 * nslices < 1, bad dtype, reps outside 1..100000), STATE (no push yet),
 * DEVICE. */
tt_status tt_stream_time_passes(tt_stream* s, const void* const* slices, int32_t nslices, tt_dtype dtype,
                                int32_t reps, float* us);

/* Description of the calling thread's last error (never NULL). */
const char* tt_last_error_string(void);

/* Library version string. */
const char* tt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TT_STREAM_H */
