// FP64 contractions launched over the whole GPU: the interface products of
// the update that are too large for the one-workgroup chain (chain_exec.hip),
// for one stream or a batch of same-shape streams, and the reconstruction of
// a slice from the cores (output conversion included).  The slice contractions that stream the whole slice live in
// pass_kernels.hip.
#include "tt_internal.h"

#include <cmath>

namespace ttk {
namespace {

// Depth groups of a wide product: a power of two with about 16 or more
// multiply-adds per group, up to 16, and up to 64 while the product's
// outputs times groups stay within 1024 blocks (deep products with few
// outputs, which would otherwise leave most of the GPU idle); a function of
// the product's shape only, the same on host and device.  A block of
// kWideThreads threads owns kWideThreads / groups consecutive outputs.
constexpr int kWideThreads = 256;
__host__ __device__ inline int depth_groups(int64_t K, int64_t nout) {
  int g = 1;
  while (g < 16 && (int64_t)g * 32 <= K) g <<= 1;
  while (g == 16 || g == 32) {
    if ((int64_t)(2 * g) * 32 > K || nout * 2 * g > (int64_t)1024 * kWideThreads) break;
    g <<= 1;
  }
  return g;
}

// Outputs per thread: JB = 4 consecutive columns j when the product asks for
// it (jb4, set by the plan) and consecutive threads run along i (A
// column-major, or B not row-major) with no operand contiguous along the depth
// only, so each A element loaded serves four outputs; else 1.  A function of
// the product's description only (host and device).
__host__ __device__ inline int wide_jb(int64_t N, int64_t ars, int64_t acs, int64_t brs, int64_t bcs, bool jb4) {
  const bool kfast = ars != 1 && bcs != 1 && (acs == 1 || brs == 1);
  const bool along_i = ars == 1 || bcs != 1;
  return (jb4 && along_i && !kfast && N >= 4) ? 4 : 1;
}

// C = A B, element strides.  Thread t of a block takes output o = base + t %
// OB (OB = 256 / groups) and the depth group t / OB (depths k = group,
// group + groups, ...); with JB = 4 output o is the run of columns
// 4 (o / M) .. +3 of row o % M.  Consecutive outputs run along i when A is
// column-major (ars == 1) and along j when it is not but B is row-major
// (bcs == 1), so the threads of one depth group read a contiguous run of one
// operand and one broadcast value of the other; when neither holds but an
// operand is contiguous along the depth (acs == 1 or brs == 1), thread t
// takes depth group t % groups of output t / groups instead, so consecutive
// threads read consecutive depths.  Each thread keeps sixteen
// loads per operand in flight (predicated at the end of its depths) and two
// accumulators; the groups' sums are added in group
// order through LDS, so the result depends on the shape only.  The block
// returns as a whole when it is past the outputs (no thread reaches the
// barrier alone).
// The JB = 4 form of wide_gemm (along i, no depth-fast operand): thread t
// computes C(i, 4 jq .. 4 jq + 3) for o = base + t % OB, i = o % M, jq = o / M,
// over the depth group t / OB, each output's terms added in the same order as
// in wide_gemm (even depths into one accumulator, odd into the other, in
// order), so the result is bitwise that of the one-output form.
__device__ __forceinline__ void wide_gemm_jb4(int64_t M, int64_t N, int64_t K, const double* A, int64_t ars,
                                              int64_t acs, const double* B, int64_t brs, int64_t bcs, double* C,
                                              int64_t crs, int64_t ccs, float* C32) {
  constexpr int JB = 4;
  __shared__ double red4[JB * kWideThreads];
  const int G = depth_groups(K, M * N), lg = __builtin_ctz(G), OB = kWideThreads >> lg, lob = __builtin_ctz(OB);
  const int64_t NJ = (N + JB - 1) / JB;
  const int64_t nout = M * NJ;
  const int64_t base = (int64_t)blockIdx.x * OB;
  if (base >= nout) return;
  const int t = threadIdx.x, ol = t & (OB - 1), g = t >> lob;
  const int64_t o = base + ol;
  const bool valid = o < nout;
  const int64_t oc = valid ? o : nout - 1;
  int64_t i, jq;
  if (nout <= INT32_MAX) {
    const uint32_t ou = (uint32_t)oc, d = (uint32_t)M;
    const uint32_t qo = ou / d;
    i = ou - qo * d;
    jq = qo;
  } else {
    i = oc % M;
    jq = oc / M;
  }
  const int64_t j0 = JB * jq;
  const double* a = A + i * ars + (int64_t)g * acs;
  const double* b[JB];
#pragma unroll
  for (int c = 0; c < JB; ++c) {
    const int64_t j = j0 + c < N ? j0 + c : N - 1;
    b[c] = B + j * bcs + (int64_t)g * brs;
  }
  const int64_t da = (int64_t)G * acs, db = (int64_t)G * brs;
  const int64_t nk = K > g ? (K - g + G - 1) >> lg : 0;
  constexpr int U = 4;  // loads in flight per operand column (even: the parity of u is that of the depth)
  double acc0[JB], acc1[JB];
#pragma unroll
  for (int c = 0; c < JB; ++c) acc0[c] = acc1[c] = 0.0;
  for (int64_t q = 0; q < nk; q += U) {
    double x[U], y[U][JB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = q + u < nk;
      x[u] = in ? a[u * da] : 0.0;
#pragma unroll
      for (int c = 0; c < JB; ++c) y[u][c] = in ? b[c][u * db] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u += 2)
#pragma unroll
      for (int c = 0; c < JB; ++c) {
        acc0[c] = fma(x[u], y[u][c], acc0[c]);
        acc1[c] = fma(x[u + 1], y[u + 1][c], acc1[c]);
      }
    a += U * da;
#pragma unroll
    for (int c = 0; c < JB; ++c) b[c] += U * db;
  }
#pragma unroll
  for (int c = 0; c < JB; ++c) red4[c * kWideThreads + t] = acc0[c] + acc1[c];
  __syncthreads();
  if (g != 0 || !valid) return;
#pragma unroll
  for (int c = 0; c < JB; ++c) {
    if (j0 + c >= N) break;
    double sum = red4[c * kWideThreads + ol];
    for (int gg = 1; gg < G; ++gg) sum += red4[c * kWideThreads + ol + OB * gg];
    const int64_t off = i * crs + (j0 + c) * ccs;
    if (C) C[off] = sum;
    if (C32) C32[off] = (float)sum;
  }
}

__device__ __forceinline__ void wide_gemm(int64_t M, int64_t N, int64_t K, const double* A, int64_t ars,
                                          int64_t acs, const double* B, int64_t brs, int64_t bcs, double* C,
                                          int64_t crs, int64_t ccs, float* C32, bool jb4) {
  if (wide_jb(N, ars, acs, brs, bcs, jb4) == 4) {
    wide_gemm_jb4(M, N, K, A, ars, acs, B, brs, bcs, C, crs, ccs, C32);
    return;
  }
  __shared__ double red[kWideThreads];
  // G and OB are powers of two: shifts and masks instead of divisions
  const int G = depth_groups(K, M * N), lg = __builtin_ctz(G), OB = kWideThreads >> lg, lob = __builtin_ctz(OB);
  const int64_t nout = M * N;
  const int64_t base = (int64_t)blockIdx.x * OB;
  if (base >= nout) return;
  // neither operand contiguous along an output index but one along the
  // depth: consecutive threads take consecutive depths instead
  const bool kfast = ars != 1 && bcs != 1 && (acs == 1 || brs == 1);
  const int t = threadIdx.x, ol = kfast ? t >> lg : t & (OB - 1), g = kfast ? t & (G - 1) : t >> lob;
  const int64_t o = base + ol;
  const bool valid = o < nout;
  const bool along_i = ars == 1 || bcs != 1;
  const int64_t oc = valid ? o : nout - 1;
  int64_t i, j;
  if (nout <= INT32_MAX) {  // 32-bit quotients (the branch is uniform)
    const uint32_t ou = (uint32_t)oc, d = (uint32_t)(along_i ? M : N);
    const uint32_t qo = ou / d, ro = ou - qo * d;
    i = along_i ? ro : qo;
    j = along_i ? qo : ro;
  } else {
    i = along_i ? oc % M : oc / N;
    j = along_i ? oc / M : oc % N;
  }
  const double* a = A + i * ars + (int64_t)g * acs;
  const double* b = B + j * bcs + (int64_t)g * brs;
  const int64_t da = (int64_t)G * acs, db = (int64_t)G * brs;
  const int64_t nk = K > g ? (K - g + G - 1) >> lg : 0;  // depths of this group
  constexpr int U = 16;  // loads in flight per operand
  double acc0 = 0.0, acc1 = 0.0;
  for (int64_t q = 0; q < nk; q += U) {
    double x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = q + u < nk;
      x[u] = in ? a[u * da] : 0.0;
      y[u] = in ? b[u * db] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u += 2) {
      acc0 = fma(x[u], y[u], acc0);
      acc1 = fma(x[u + 1], y[u + 1], acc1);
    }
    a += U * da;
    b += U * db;
  }
  red[t] = acc0 + acc1;
  __syncthreads();
  if (g != 0 || !valid) return;
  double sum = red[kfast ? ol * G : ol];
  for (int gg = 1; gg < G; ++gg) sum += red[kfast ? ol * G + gg : ol + OB * gg];
  if (C) C[i * crs + j * ccs] = sum;
  if (C32) C32[i * crs + j * ccs] = (float)sum;
}

__global__ void __launch_bounds__(kWideThreads) k_gemm64(int64_t M, int64_t N, int64_t K, const double* A,
                                                         int64_t ars, int64_t acs, const double* B, int64_t brs,
                                                         int64_t bcs, double* C, int64_t crs, int64_t ccs,
                                                         float* C32) {
  wide_gemm(M, N, K, A, ars, acs, B, brs, bcs, C, crs, ccs, C32, false);
}

typedef const TT_CONSTANT_AS ChainOp ConstChainOp;
typedef const TT_CONSTANT_AS uint64_t ConstWord;

// The same product for the GEMM *ops[blockIdx.y] of a batch; blocks past the
// product's own outputs return.  The op pointers and ops are read-only during
// the launch; reading them through the constant address space keeps the
// descriptor in scalar registers.
__global__ void __launch_bounds__(kWideThreads) k_gemm64_ops(const ChainOp* const* __restrict__ ops) {
  const uint64_t addr = ((ConstWord*)(const void*)ops)[blockIdx.y];
  const ChainOp op = *(ConstChainOp*)addr;
  wide_gemm(op.m, op.n, op.k, op.a, op.ars, op.acs, op.b, op.brs, op.bcs, op.c, op.crs, op.ccs, op.c32,
            op.rho == kWideJb4);
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

int64_t gemm64_blocks(int64_t M, int64_t N, int64_t K, int64_t ars, int64_t acs, int64_t brs, int64_t bcs,
                      bool jb4) {
  if (M <= 0 || N <= 0) return 0;
  const int64_t ob = kWideThreads / depth_groups(K, M * N);
  const int jb = wide_jb(N, ars, acs, brs, bcs, jb4);
  return (M * ((N + jb - 1) / jb) + ob - 1) / ob;
}

hipError_t gemm64(hipStream_t st, int64_t M, int64_t N, int64_t K,
                  const double* A, int64_t ars, int64_t acs,
                  const double* B, int64_t brs, int64_t bcs,
                  double* C, int64_t crs, int64_t ccs, float* C32) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t blocks = gemm64_blocks(M, N, K, ars, acs, brs, bcs, false);
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm64, dim3((unsigned)blocks), dim3(kWideThreads), 0, st, M, N, K, A, ars, acs, B, brs,
                     bcs, C, crs, ccs, C32);
  return hipGetLastError();
}

hipError_t gemm64_ops(hipStream_t st, const ChainOp* const* ops_dev, int nops, int64_t gx) {
  if (nops == 0 || gx == 0) return hipSuccess;
  if (nops < 0 || nops > 65535 || gx > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm64_ops, dim3((unsigned)gx, nops), dim3(kWideThreads), 0, st, ops_dev);
  return hipGetLastError();
}

hipError_t convert_out(hipStream_t st, const double* src, void* dst, tt_dtype dt, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_out, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, src, dst, (int)dt, n);
  return hipGetLastError();
}

}  // namespace ttk
