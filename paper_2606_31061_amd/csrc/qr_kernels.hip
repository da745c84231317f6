// Thin Householder QR (FP64) of the small tall matrices that re-orthogonalise
// the cores in every update: the forward sweep's QR of the (r_{k-1} I_k) x r_k
// local solution and the LQ sweep's QR of the transposed r_{k-1} x (I_k r_k)
// unfolding (Algorithm 1).  Up to 768 rows and 64 columns.
//
// One workgroup of 16 waves.  Column c belongs to wave c mod 16 and lives in
// that wave's registers for the whole factorisation (row i in lane i mod 64,
// slot i / 64).  Step j: the owner of column j builds the reflector
// H_j = I - tau v v^T (v_j = 1) and publishes v and tau in LDS; after one
// barrier every wave applies H_j to its own columns, each dot product being a
// wave reduction done with DPP lane moves.  The explicit thin Q is then formed
// by applying H_{n-1} .. H_0 to the unit columns; that phase reads only LDS
// and needs no barrier.  Signs are fixed so that diag(R) >= 0, and a column
// whose remaining norm is <= tol ||M||_F gets the identity in place of a
// reflector (R_jj = 0), as in the oracle.
#include "tt_internal.h"

namespace ttk {
namespace {

constexpr int kWaves = 16;

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes; every lane gets the same (bitwise) result.  Lanes
// exchange within quads (xor 1, xor 2), then across half rows and rows of 16
// by mirroring, and the four row sums are combined in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  const double a = read_lane(v, 0), b = read_lane(v, 16), c = read_lane(v, 32), d = read_lane(v, 48);
  return (a + b) + (c + d);
}

// S = rows per lane (m <= 64 S), C = columns per wave (n <= 16 C).
template <int S, int C>
__global__ void __launch_bounds__(kWaves * 64) k_qr_reg(int m, int n, const double* __restrict__ M, int64_t mrs,
                                                       int64_t mcs, double* __restrict__ Q, int64_t qrs,
                                                       int64_t qcs, double* __restrict__ R, double tol) {
  extern __shared__ double lds[];
  double* V = lds;                 // m x n reflectors, column-major
  double* tau = V + (size_t)m * n; // n
  double* beta = tau + n;          // n
  double* red = beta + n;          // kWaves
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

  double a[C][S];
  // load owned columns and the Frobenius norm
  double ss = 0.0;
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const int c = w + kWaves * u;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = lane + 64 * s;
      double x = 0.0;
      if (c < n && i < m) x = M[i * mrs + c * mcs];
      a[u][s] = x;
      ss = fma(x, x, ss);
    }
  }
  ss = wave_sum(ss);
  if (lane == 0) red[w] = ss;
  __syncthreads();
  double fro2 = 0.0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) fro2 += red[i];
  const double thr = tol * sqrt(fro2);

  // ---- factorisation
  for (int j = 0; j < n; ++j) {
    const int ow = j % kWaves, uj = j / kWaves;
    if (w == ow) {
      double nn = 0.0, alpha = 0.0;
#pragma unroll
      for (int u = 0; u < C; ++u) {
        if (u != uj) continue;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int i = lane + 64 * s;
          const double x = (i >= j && i < m) ? a[u][s] : 0.0;
          nn = fma(x, x, nn);
        }
        double xj = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s)
          if (s == j / 64) xj = a[u][s];
        alpha = read_lane(xj, j % 64);
      }
      nn = wave_sum(nn);
      const double nrm = sqrt(nn);
#pragma unroll
      for (int u = 0; u < C; ++u) {
        if (u != uj) continue;
        if (!(nrm > thr)) {
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const int i = lane + 64 * s;
            if (i >= j && i < m) a[u][s] = 0.0;
            if (i > j && i < m) V[i + (size_t)j * m] = 0.0;
          }
          if (lane == 0) { tau[j] = 0.0; beta[j] = 0.0; }
        } else {
          const double b = alpha >= 0.0 ? -nrm : nrm;
          const double scal = 1.0 / (alpha - b);
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const int i = lane + 64 * s;
            if (i > j && i < m) {
              const double v = a[u][s] * scal;
              a[u][s] = v;
              V[i + (size_t)j * m] = v;
            } else if (i == j) {
              a[u][s] = b;
            }
          }
          if (lane == 0) { tau[j] = (b - alpha) / b; beta[j] = b; }
        }
      }
    }
    __syncthreads();
    const double t = tau[j];
    if (t == 0.0) continue;
    double v[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = lane + 64 * s;
      v[s] = (i > j && i < m) ? V[i + (size_t)j * m] : (i == j ? 1.0 : 0.0);
    }
    double d[C];
#pragma unroll
    for (int u = 0; u < C; ++u) {
      double p = 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s) p = fma(v[s], a[u][s], p);
      d[u] = p;
    }
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int c = w + kWaves * u;
      if (c > j && c < n) d[u] = wave_sum(d[u]);
    }
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int c = w + kWaves * u;
      if (c <= j || c >= n) continue;
      const double tw = t * d[u];
#pragma unroll
      for (int s = 0; s < S; ++s) a[u][s] = fma(-tw, v[s], a[u][s]);
    }
  }
  __syncthreads();

  // ---- R (rows < n of the owned columns; diagonal = beta), signs diag(R) >= 0
  if (R) {
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int c = w + kWaves * u;
      if (c >= n) continue;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int i = lane + 64 * s;
        if (i < n) {
          const double sg = beta[i] < 0.0 ? -1.0 : 1.0;
          R[i + (size_t)c * n] = (i <= c) ? sg * a[u][s] : 0.0;
        }
      }
    }
  }

  // ---- explicit Q: start from the unit columns, apply H_{n-1} .. H_0
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const int c = w + kWaves * u;
#pragma unroll
    for (int s = 0; s < S; ++s) a[u][s] = (lane + 64 * s == c) ? 1.0 : 0.0;
  }
  for (int j = n - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t == 0.0) continue;
    double v[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = lane + 64 * s;
      v[s] = (i > j && i < m) ? V[i + (size_t)j * m] : (i == j ? 1.0 : 0.0);
    }
    double d[C];
#pragma unroll
    for (int u = 0; u < C; ++u) {
      double p = 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s) p = fma(v[s], a[u][s], p);
      d[u] = p;
    }
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int c = w + kWaves * u;
      if (c >= j && c < n) d[u] = wave_sum(d[u]);
    }
#pragma unroll
    for (int u = 0; u < C; ++u) {
      const int c = w + kWaves * u;
      if (c < j || c >= n) continue;
      const double tw = t * d[u];
#pragma unroll
      for (int s = 0; s < S; ++s) a[u][s] = fma(-tw, v[s], a[u][s]);
    }
  }
#pragma unroll
  for (int u = 0; u < C; ++u) {
    const int c = w + kWaves * u;
    if (c >= n) continue;
    const double sg = beta[c] < 0.0 ? -1.0 : 1.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = lane + 64 * s;
      if (i < m) Q[i * qrs + c * qcs] = sg * a[u][s];
    }
  }
}

template <int S, int C>
hipError_t launch_reg(hipStream_t st, int m, int n, const double* M, int64_t mrs, int64_t mcs, double* Q,
                      int64_t qrs, int64_t qcs, double* R, double tol) {
  const size_t lds = ((size_t)m * n + 2 * n + kWaves) * sizeof(double);
  hipLaunchKernelGGL((k_qr_reg<S, C>), dim3(1), dim3(kWaves * 64), lds, st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
  return hipGetLastError();
}

template <int S>
hipError_t dispatch_c(hipStream_t st, int m, int n, const double* M, int64_t mrs, int64_t mcs, double* Q, int64_t qrs,
                      int64_t qcs, double* R, double tol) {
  if (n <= 16) return launch_reg<S, 1>(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
  if (n <= 32) return launch_reg<S, 2>(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
  return launch_reg<S, 4>(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
}

template <int S, int C>
hipError_t set_attr(size_t lds) {
  return hipFuncSetAttribute((const void*)k_qr_reg<S, C>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace

// Largest matrix the register kernel takes: 768 rows (S = 12 slots) and, with
// 12 slots, 32 columns; with at most 512 rows, 64 columns.  The LDS must hold
// the m x n reflectors.
bool qr_reg_fits(int m, int n, size_t lds_limit) {
  if (m < n || n < 1 || n > 64 || m > 768) return false;
  if (m > 512 && n > 32) return false;
  return ((size_t)m * n + 2 * n + kWaves) * sizeof(double) <= lds_limit;
}

hipError_t qr_reg(hipStream_t st, int m, int n, const double* M, int64_t mrs, int64_t mcs, double* Q, int64_t qrs,
                  int64_t qcs, double* R, double tol) {
  if (m <= 64) return dispatch_c<1>(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
  if (m <= 128) return dispatch_c<2>(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
  if (m <= 256) return dispatch_c<4>(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
  if (m <= 512) return dispatch_c<8>(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
  if (n <= 16) return launch_reg<12, 1>(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
  return launch_reg<12, 2>(st, m, n, M, mrs, mcs, Q, qrs, qcs, R, tol);
}

hipError_t qr_reg_setup(size_t lds) {
  hipError_t e = hipSuccess;
#define TT_ATTR(S, C) \
  if (e == hipSuccess) e = set_attr<S, C>(lds);
  TT_ATTR(1, 1) TT_ATTR(1, 2) TT_ATTR(1, 4) TT_ATTR(2, 1) TT_ATTR(2, 2) TT_ATTR(2, 4) TT_ATTR(4, 1) TT_ATTR(4, 2)
  TT_ATTR(4, 4) TT_ATTR(8, 1) TT_ATTR(8, 2) TT_ATTR(8, 4) TT_ATTR(12, 1) TT_ATTR(12, 2)
#undef TT_ATTR
  return e;
}

}  // namespace ttk
