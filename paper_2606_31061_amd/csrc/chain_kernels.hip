// FP64 kernels of the update's small chain: thin Householder QR / LQ (the
// gauge re-orthogonalisation of Algorithm 1), the small interface
// contractions, normalisation of the temporal vector and the state commit.
// These are latency-bound (operands of at most a few hundred KB); the slice
// contractions that stream the whole slice live in pass_kernels.hip.
#include "tt_internal.h"

#include <cmath>

namespace ttk {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup; every thread receives the total.  Fixed reduction
// order, so the result is reproducible run to run.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  return s;
}

// Householder factorisation of the m x n column-major matrix A (leading
// dimension lda) by one workgroup.  On exit R is on and above the diagonal,
// the reflector vectors (unit leading entry implied) below it, tau[j] their
// scalars: H_j = I - tau_j v_j v_j^T with H_j x = beta e_1, beta = -sign(x_1)||x||.
// A column whose remaining norm is <= thr gets tau = 0 and is zeroed from the
// diagonal down (identity reflector, R_jj = 0).
template <int NT>
__device__ void hh_factor(double* A, int m, int n, int lda, double thr, double* tau, double* red) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int j = 0; j < n; ++j) {
    double* cj = A + (int64_t)j * lda;
    double p = 0.0;
    for (int i = j + tid; i < m; i += NT) { const double x = cj[i]; p = fma(x, x, p); }
    const double nrm2 = block_sum<NT>(p, red);
    const double alpha = cj[j];
    const double nrm = sqrt(nrm2);
    __syncthreads();
    if (!(nrm > thr)) {
      for (int i = j + tid; i < m; i += NT) cj[i] = 0.0;
      if (tid == 0) tau[j] = 0.0;
      __syncthreads();
      continue;
    }
    const double beta = alpha >= 0.0 ? -nrm : nrm;
    const double scal = 1.0 / (alpha - beta);
    for (int i = j + 1 + tid; i < m; i += NT) cj[i] *= scal;
    const double t = (beta - alpha) / beta;
    __syncthreads();
    if (tid == 0) { cj[j] = beta; tau[j] = t; }
    // Apply H_j to the trailing columns: one wave per column.
    for (int c = j + 1 + wid; c < n; c += NW) {
      double* cc = A + (int64_t)c * lda;
      double d = (lane == 0) ? cc[j] : 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) d = fma(cj[i], cc[i], d);
      d = wave_sum(d);
      const double tw = t * d;
      if (lane == 0) cc[j] -= tw;
      for (int i = j + 1 + lane; i < m; i += 64) cc[i] = fma(-tw, cj[i], cc[i]);
    }
    __syncthreads();
  }
}

// Overwrite the factored A with the explicit thin Q = H_0 ... H_{n-1} [I; 0]
// (backward accumulation), then flip column j when sgn[j] < 0.
template <int NT>
__device__ void hh_form_q(double* A, int m, int n, int lda, const double* tau, const double* sgn) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int j = n - 1; j >= 0; --j) {
    const double t = tau[j];
    double* cj = A + (int64_t)j * lda;
    if (t != 0.0) {
      for (int c = j + 1 + wid; c < n; c += NW) {
        double* cc = A + (int64_t)c * lda;
        double d = (lane == 0) ? cc[j] : 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) d = fma(cj[i], cc[i], d);
        d = wave_sum(d);
        const double tw = t * d;
        if (lane == 0) cc[j] -= tw;
        for (int i = j + 1 + lane; i < m; i += 64) cc[i] = fma(-tw, cj[i], cc[i]);
      }
    }
    __syncthreads();
    for (int i = tid; i < m; i += NT) {
      double v;
      if (i < j) v = 0.0;
      else if (i == j) v = 1.0 - t;
      else v = -t * cj[i];
      cj[i] = v;
    }
    __syncthreads();
  }
  for (int j = 0; j < n; ++j) {
    if (sgn[j] < 0.0) {
      double* cj = A + (int64_t)j * lda;
      for (int i = tid; i < m; i += NT) cj[i] = -cj[i];
    }
  }
  __syncthreads();
}

template <int NT>
__device__ void qr_body(double* W, int m, int n, const double* M, int64_t mrs, int64_t mcs,
                        double* Q, int64_t qrs, int64_t qcs, double* R, double tol,
                        double* tau, double* sgn, double* red) {
  const int tid = threadIdx.x;
  // load and Frobenius norm
  double p = 0.0;
  const int64_t total = (int64_t)m * n;
  for (int64_t e = tid; e < total; e += NT) {
    const int i = (int)(e % m), j = (int)(e / m);
    const double x = M[i * mrs + j * mcs];
    W[e] = x;
    p = fma(x, x, p);
  }
  const double fro = sqrt(block_sum<NT>(p, red));
  hh_factor<NT>(W, m, n, m, tol * fro, tau, red);
  for (int j = tid; j < n; j += NT) sgn[j] = (W[j + (int64_t)j * m] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  if (R) {
    for (int e = tid; e < n * n; e += NT) {
      const int i = e % n, j = e / n;
      R[e] = (i <= j) ? sgn[i] * W[i + (int64_t)j * m] : 0.0;
    }
  }
  __syncthreads();
  hh_form_q<NT>(W, m, n, m, tau, sgn);
  for (int64_t e = tid; e < total; e += NT) {
    const int i = (int)(e % m), j = (int)(e / m);
    Q[i * qrs + j * qcs] = W[e];
  }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_qr64_lds(int m, int n, const double* M, int64_t mrs, int64_t mcs,
                                                 double* Q, int64_t qrs, int64_t qcs, double* R, double tol) {
  extern __shared__ double smem[];
  double* tau = smem;
  double* sgn = tau + n;
  double* red = sgn + n;
  double* W = red + 32;
  qr_body<NT>(W, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol, tau, sgn, red);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_qr64_glb(int m, int n, const double* M, int64_t mrs, int64_t mcs,
                                                 double* Q, int64_t qrs, int64_t qcs, double* R, double tol,
                                                 double* gwork) {
  extern __shared__ double smem[];
  double* tau = smem;
  double* sgn = tau + n;
  double* red = sgn + n;
  qr_body<NT>(gwork, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol, tau, sgn, red);
}

// Split-K FP64 GEMM: KS consecutive lanes share one output element.
__global__ void __launch_bounds__(256) k_gemm64(int64_t M, int64_t N, int64_t K, int ks,
                                                const double* __restrict__ A, int64_t ars, int64_t acs,
                                                const double* __restrict__ B, int64_t brs, int64_t bcs,
                                                double* C, int64_t crs, int64_t ccs, float* C32) {
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int q = (int)(gt % ks);
  const int64_t out = gt / ks;
  const bool valid = out < M * N;
  const int64_t i = valid ? out % M : 0, j = valid ? out / M : 0;
  double acc = 0.0;
  if (valid) {
    const double* a = A + i * ars;
    const double* b = B + j * bcs;
    for (int64_t k = q; k < K; k += ks) acc = fma(a[k * acs], b[k * brs], acc);
  }
  for (int o = ks >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (valid && q == 0) {
    C[i * crs + j * ccs] = acc;
    if (C32) C32[i * crs + j * ccs] = (float)acc;
  }
}

__global__ void k_copy64(double* dst, const double* src, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

__global__ void __launch_bounds__(256) k_normalize_g(const double* g_in, double* g_out, int rm,
                                                     const double* Gm_in, double* Gm_out, int64_t gm_len) {
  __shared__ double red[8];
  double p = 0.0;
  for (int i = threadIdx.x; i < rm; i += 256) p = fma(g_in[i], g_in[i], p);
  const double nu = sqrt(block_sum<256>(p, red));
  if (nu > 0.0) {
    const double inv = 1.0 / nu;
    for (int i = threadIdx.x; i < rm; i += 256) g_out[i] = g_in[i] * inv;
    for (int64_t e = threadIdx.x; e < gm_len; e += 256) Gm_out[e] = Gm_in[e] * nu;
  } else {
    for (int i = threadIdx.x; i < rm; i += 256) g_out[i] = (i == 0) ? 1.0 : 0.0;
    for (int64_t e = threadIdx.x; e < gm_len; e += 256) Gm_out[e] = Gm_in[e];
  }
}

// Commit, part 1: every block copies its share of the new state (and the
// temporal row) when the update saw a finite slice.
__global__ void __launch_bounds__(256) k_commit_copy(const int* flag, const double* new_state, double* master,
                                                     int64_t len, const double* g_new, int rm, double* history,
                                                     int64_t hist_cap, const int64_t* t_dev) {
  if (*flag != 0) return;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x)
    master[e] = new_state[e];
  if (blockIdx.x == 0 && history && hist_cap > 0) {
    const int64_t row = (*t_dev) % hist_cap;
    for (int i = threadIdx.x; i < rm; i += blockDim.x) history[row * rm + i] = g_new[i];
  }
}

// Commit, part 2: advance t (or count the rejected slice) and clear the flag.
__global__ void k_commit_final(int* flag, int64_t* t_dev, int* rejected) {
  if (threadIdx.x == 0) {
    if (*flag == 0) *t_dev += 1;
    else *rejected += 1;
    *flag = 0;
  }
}

__global__ void k_to_f32(const double* src, float* dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

__global__ void k_convert_out(const double* src, void* dst, int dt, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    if (dt == TT_F64) static_cast<double*>(dst)[e] = src[e];
    else static_cast<float*>(dst)[e] = (float)src[e];
  }
}

inline unsigned grid_for(int64_t work, int threads, int64_t cap = 65536) {
  int64_t b = (work + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

}  // namespace

hipError_t gemm64(hipStream_t st, int64_t M, int64_t N, int64_t K,
                  const double* A, int64_t ars, int64_t acs,
                  const double* B, int64_t brs, int64_t bcs,
                  double* C, int64_t crs, int64_t ccs, float* C32) {
  if (M <= 0 || N <= 0) return hipSuccess;
  int ks = 1;
  while (ks < 64 && (int64_t)ks * 8 < K) ks <<= 1;
  const int64_t threads = M * N * ks;
  const int64_t blocks = (threads + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm64, dim3((unsigned)blocks), dim3(256), 0, st, M, N, K, ks, A, ars, acs, B, brs, bcs,
                     C, crs, ccs, C32);
  return hipGetLastError();
}

bool qr_reg_fits(int m, int n, size_t lds_limit);
hipError_t qr_reg(hipStream_t st, int m, int n, const double* M, int64_t mrs, int64_t mcs, double* Q, int64_t qrs,
                  int64_t qcs, double* R, double tol);
hipError_t qr_reg_setup(size_t lds);

hipError_t qr64(hipStream_t st, int m, int n, const double* M, int64_t mrs, int64_t mcs,
                double* Q, int64_t qrs, int64_t qcs, double* R, double tol,
                double* gwork, size_t lds_limit) {
  if (m < n || n < 1) return hipErrorInvalidValue;
  if (qr_reg_fits(m, n, lds_limit)) return qr_reg(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
  const size_t small = (size_t)(2 * n + 32) * sizeof(double);
  const size_t need = small + (size_t)m * n * sizeof(double);
  if (need <= lds_limit) {
    hipLaunchKernelGGL(k_qr64_lds<kQrThreads>, dim3(1), dim3(kQrThreads), need, st, m, n, M, mrs, mcs, Q, qrs, qcs,
                       R, tol);
  } else {
    hipLaunchKernelGGL(k_qr64_glb<kQrThreads>, dim3(1), dim3(kQrThreads), small, st, m, n, M, mrs, mcs, Q, qrs,
                       qcs, R, tol, gwork);
  }
  return hipGetLastError();
}

hipError_t copy64(hipStream_t st, double* dst, const double* src, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

hipError_t normalize_g(hipStream_t st, const double* g_in, double* g_out, int rm,
                       const double* Gm_in, double* Gm_out, int64_t gm_len) {
  hipLaunchKernelGGL(k_normalize_g, dim3(1), dim3(256), 0, st, g_in, g_out, rm, Gm_in, Gm_out, gm_len);
  return hipGetLastError();
}

hipError_t commit(hipStream_t st, int* flag, const double* new_state, double* master, int64_t len,
                  const double* g_new, int rm, double* history, int64_t hist_cap,
                  int64_t* t_dev, int* rejected) {
  hipLaunchKernelGGL(k_commit_copy, dim3(grid_for(len, 256, 256)), dim3(256), 0, st, flag, new_state, master, len,
                     g_new, rm, history, hist_cap, t_dev);
  hipLaunchKernelGGL(k_commit_final, dim3(1), dim3(64), 0, st, flag, t_dev, rejected);
  return hipGetLastError();
}

hipError_t convert_out(hipStream_t st, const double* src, void* dst, tt_dtype dt, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_out, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, src, dst, (int)dt, n);
  return hipGetLastError();
}

hipError_t to_f32(hipStream_t st, const double* src, float* dst, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

// Needed once per process before launching a kernel with more than 64 KB of
// dynamic LDS.
hipError_t qr64_setup(size_t lds_limit) {
  hipError_t e = hipFuncSetAttribute((const void*)k_qr64_lds<kQrThreads>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit);
  if (e != hipSuccess) return e;
  return qr_reg_setup(lds_limit);
}

}  // namespace ttk
