/*
 * tt_kernels.h - the update's building blocks as separate C entry points.
 *
 * These expose, one at a time, the device kernels that tt_stream_push_slice
 * chains together, so that each can be checked or reused on its own.  All
 * pointers are HIP device pointers; `hip_stream` is a hipStream_t (NULL = the
 * default stream).  Every call is stream-ordered and returns before the work
 * completes.  Matrices are column-major (first index fastest).  Errors:
 * TT_ERR_INVALID_ARG for null pointers or sizes out of range, TT_ERR_DEVICE if
 * a launch fails.  The caller owns every buffer.
 */
#ifndef TT_KERNELS_H
#define TT_KERNELS_H

#include "tt_stream.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Pass 1 of an update (Eq. 5 for the cores k <= k*, contracted with the right
 * interface first): Z = X B^T for the P x J slice unfolding X (element type
 * x_dtype), B r x J FP32, Z P x r FP64.  1 <= r <= 64.  workspace (device,
 * caller-owned, no initialisation needed) must hold
 * tt_kernel_pass1_workspace(P, J, r) bytes; it receives the FP32 partial
 * tiles, which are then added in FP64 in a fixed order. */
tt_status tt_kernel_pass1(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r,
                          const float* B, double* Z, void* workspace, int32_t* nonfinite_flag,
                          void* hip_stream);
size_t tt_kernel_pass1_workspace(int64_t P, int64_t J, int32_t r);

/* tt_kernel_pass1 without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the FP32 partial tiles go to a static
 * device array of tt_kernel_pass1_noalloc_max() bytes (32 MiB) that the
 * library holds on every GPU it runs on until the process ends.  Same
 * arguments, kernels, launch plan and results (bit for bit) as
 * tt_kernel_pass1; it allocates nothing.  All calls on one GPU share that
 * GPU's array: calls whose work overlaps on one GPU (different HIP streams,
 * or host threads) race on it and must be serialised by the caller (calls on
 * one HIP stream are ordered).  Nothing in the array needs clearing: every
 * partial tile is written before it is read.  Errors: as tt_kernel_pass1,
 * plus TT_ERR_UNSUPPORTED when tt_kernel_pass1_workspace(P, J, r) exceeds
 * tt_kernel_pass1_noalloc_max() (e.g. 1080 x 5760 slices at r = 32 need
 * 13 MB), and TT_ERR_DEVICE if the array's device address cannot be found. */
tt_status tt_kernel_pass1_noalloc(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r,
                                  const float* B, double* Z, int32_t* nonfinite_flag, void* hip_stream);
size_t tt_kernel_pass1_noalloc_max(void);

/* Pass 2 of an update (Eq. 5 for the cores k > k*, contracted with the left
 * interface first): Y = A^T X, A P x r FP32, Y r x J FP64.  1 <= r <= 64. */
tt_status tt_kernel_pass2(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r,
                          const float* A, double* Y, int32_t* nonfinite_flag, void* hip_stream);

/* BF16-input, FP32-accumulate variants of the two passes (the reduced-
 * precision option of the contractions; the QR and Gram steps of Section 3.4
 * stay FP64): every element of X (any x_dtype) and of the interface is
 * rounded to BF16 (round to nearest even), products are accumulated in FP32
 * per tile (a block's waves added in wave order) and, where a tile's
 * reduction is split over blocks, the partial tiles are added in FP64 in a
 * fixed order.
 * Same shapes, layouts and flag as tt_kernel_pass1 / tt_kernel_pass2; the
 * result does not depend on block timing.  The workspace (device, caller-
 * owned, at least the size returned by the matching _workspace function, no
 * initialisation needed) receives FP32 partial tiles.  A slice value beyond
 * the BF16 range becomes infinite and sets the flag. */
size_t tt_kernel_pass1_bf16_workspace(int64_t P, int64_t J, int32_t r);
tt_status tt_kernel_pass1_bf16(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r,
                               const float* B, double* Z, void* workspace, int32_t* nonfinite_flag,
                               void* hip_stream);
size_t tt_kernel_pass2_bf16_workspace(int64_t P, int64_t J, int32_t r);
tt_status tt_kernel_pass2_bf16(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r,
                               const float* A, double* Y, void* workspace, int32_t* nonfinite_flag,
                               void* hip_stream);
/* Thin QR of an m x n FP64 matrix (m >= n >= 1, n <= 256) as used to
 * re-orthogonalise a core (Algorithm 1; Section 3.4.2): M = Q R, Q^T Q = I,
 * diag(R) >= 0.  Well-conditioned matrices with n <= 32 take CholeskyQR2
 * (two Gram/Cholesky passes); otherwise, or when a Cholesky pivot falls below
 * (1e-6 ||M||_F)^2, Householder, where a column whose remaining norm is
 * <= 64 eps ||M||_F gets the identity reflector (R_jj = 0).  M, Q column-major
 * with leading dimension m (Q may alias M); R n x n (may be NULL).
 * workspace must hold m*n doubles.  TT_ERR_UNSUPPORTED for n > 256. */
tt_status tt_kernel_qr(int32_t m, int32_t n, const double* M, double* Q, double* R,
                       double* workspace, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* TT_KERNELS_H */
