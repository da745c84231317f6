// Internal declarations shared by the runtime and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstdint>

#include "tt_stream.h"

namespace ttk {

// Records `msg` as the calling thread's last error and returns `st`.
tt_status set_error(tt_status st, const char* msg);

// Threads of the one-workgroup FP64 factorisation kernels.
constexpr int kQrThreads = 256;
// Rows of the slice staged per wave in pass 2 (multiple of 8).
constexpr int kPass2SlabMax = 72;
constexpr int kPass2Waves = 8;

// ---------------------------------------------------------------- chain (FP64)
// C(i,j) = sum_k A(i,k) B(k,j) with element strides; optional FP32 copy of C.
hipError_t gemm64(hipStream_t st, int64_t M, int64_t N, int64_t K,
                  const double* A, int64_t ars, int64_t acs,
                  const double* B, int64_t brs, int64_t bcs,
                  double* C, int64_t crs, int64_t ccs, float* C32);

// Thin Householder QR of an m x n matrix M (element (i,j) at M[i*mrs + j*mcs]).
// Writes Q (m x n) at Q[i*qrs + j*qcs]; if R != nullptr writes R (n x n,
// column-major, leading dimension n).  diag(R) >= 0; a column whose remaining
// norm is <= tol*||M||_F gets the identity reflector (R_jj = 0).  gwork holds
// m*n doubles when the matrix does not fit in LDS.  The input may alias Q.
hipError_t qr64(hipStream_t st, int m, int n, const double* M, int64_t mrs, int64_t mcs,
                double* Q, int64_t qrs, int64_t qcs, double* R, double tol,
                double* gwork, size_t lds_limit);

// dst[i] = src[i] * (*scale_src) if scale_src else src[i]; count n.
hipError_t copy64(hipStream_t st, double* dst, const double* src, int64_t n);

// g normalisation (Section 3.4.1): nu = ||g||; if nu > 0: Gm_out = nu * Gm_in,
// g_out = g_in / nu; else g_out = e_1 and Gm_out = Gm_in.
hipError_t normalize_g(hipStream_t st, const double* g_in, double* g_out, int rm,
                       const double* Gm_in, double* Gm_out, int64_t gm_len);

// Commit: if *flag == 0 copy new state (len doubles) into master, append g to
// the history ring and advance t; else count a rejected update.
hipError_t commit(hipStream_t st, int* flag, const double* new_state, double* master, int64_t len,
                  const double* g_new, int rm, double* history, int64_t hist_cap,
                  int64_t* t_dev, int* rejected);

// Element conversion FP64 -> out dtype (F64/F32).
hipError_t convert_out(hipStream_t st, const double* src, void* dst, tt_dtype dt, int64_t n);

// Host slice (F64/F32/BF16) already on device: nonfinite scan not needed (passes flag it).

// ---------------------------------------------------------------- passes (FP32)
// Pass 1: Z(p,a) = sum_j X(p,j) B(a,j), X P x J (p fastest) of dtype `xdt`,
// B r x J FP32; Z written FP64 (P x r column-major) from FP32 partial tiles
// (ws, plan.ws_floats floats) added in FP64.  Sets *flag if Z is non-finite.
struct Pass1Plan {
  int vec = 1;        // rows per lane (row tile = 32 vec)
  int ntn = 1;        // 32-column MFMA tiles of the rank (r <= 32 ntn)
  int waves = 8;      // waves per block
  int tiles = 1;      // row tiles
  int chunks = 1;     // column chunks
  size_t ws_floats = 0;
};
Pass1Plan pass1_plan(int64_t P, int64_t J, int r, int cus);
// Recomputes tiles and ws_floats after vec/ntn/waves/chunks were set.
Pass1Plan finish_plan(Pass1Plan plan, int64_t P);
hipError_t pass1(hipStream_t st, const void* X, tt_dtype xdt, const Pass1Plan& plan, int64_t P, int64_t J, int r,
                 const float* B, double* Z, float* ws, int* flag);

// Pass 2: Y(a,j) = sum_p A(p,a) X(p,j); A P x r FP32 column-major; Y FP64
// r x J column-major.  Sets *flag if Y non-finite.
hipError_t pass2(hipStream_t st, const void* X, tt_dtype xdt, int64_t P, int64_t J, int r,
                 const float* A, double* Y, int* flag);

// Reconstruction of the latest slice: out = G_1 x ... x G_m x g (FP64 chain).
// Implemented on the runtime side with gemm64.

}  // namespace ttk
