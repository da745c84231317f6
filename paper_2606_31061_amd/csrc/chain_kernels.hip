// FP64 contractions launched over the whole GPU: the interface products of
// the update that are too large for the one-workgroup chain (chain_exec.hip),
// for one stream or a batch of same-shape streams, and the reconstruction of
// a slice from the cores (output conversion included).  The slice contractions that stream the whole slice live in
// pass_kernels.hip.
#include "tt_internal.h"

#include <cmath>

namespace ttk {
namespace {

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
    if (C) C[i * crs + j * ccs] = acc;
    if (C32) C32[i * crs + j * ccs] = (float)acc;
  }
}

typedef const TT_CONSTANT_AS ChainOp ConstChainOp;
typedef const TT_CONSTANT_AS uint64_t ConstWord;

// Lanes sharing one output element: the depth split of an M x N x K product
// (a function of K only, the same on host and device).
__host__ __device__ inline int depth_split(int64_t K) {
  int ks = 1;
  while (ks < 64 && (int64_t)ks * 8 < K) ks <<= 1;
  return ks;
}

// The same product for the GEMM *ops[blockIdx.y] of a batch; blocks past the
// product's own grid return.  The op pointers and ops are read-only during
// the launch; reading them through the constant address space keeps the
// descriptor in scalar registers.
__global__ void __launch_bounds__(256) k_gemm64_ops(const ChainOp* const* __restrict__ ops) {
  const uint64_t addr = ((ConstWord*)(const void*)ops)[blockIdx.y];
  const ChainOp op = *(ConstChainOp*)addr;
  const int64_t M = op.m, N = op.n, K = op.k;
  const int ks = depth_split(K);
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int q = (int)(gt % ks);
  const int64_t out = gt / ks;
  if (blockIdx.x * (int64_t)blockDim.x >= M * N * ks) return;
  const bool valid = out < M * N;
  const int64_t i = valid ? out % M : 0, j = valid ? out / M : 0;
  double acc = 0.0;
  if (valid) {
    const double* a = op.a + i * op.ars;
    const double* b = op.b + j * op.bcs;
    for (int64_t k = q; k < K; k += ks) acc = fma(a[k * op.acs], b[k * op.brs], acc);
  }
  for (int o = ks >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (valid && q == 0) {
    if (op.c) op.c[i * op.crs + j * op.ccs] = acc;
    if (op.c32) op.c32[i * op.crs + j * op.ccs] = (float)acc;
  }
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
  const int ks = depth_split(K);
  const int64_t threads = M * N * ks;
  const int64_t blocks = (threads + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm64, dim3((unsigned)blocks), dim3(256), 0, st, M, N, K, ks, A, ars, acs, B, brs, bcs,
                     C, crs, ccs, C32);
  return hipGetLastError();
}

int64_t gemm64_blocks(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0) return 0;
  return (M * N * depth_split(K) + 255) / 256;
}

hipError_t gemm64_ops(hipStream_t st, const ChainOp* const* ops_dev, int nops, int64_t gx) {
  if (nops == 0 || gx == 0) return hipSuccess;
  if (nops < 0 || nops > 65535 || gx > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm64_ops, dim3((unsigned)gx, nops), dim3(256), 0, st, ops_dev);
  return hipGetLastError();
}

hipError_t convert_out(hipStream_t st, const double* src, void* dst, tt_dtype dt, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_out, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, src, dst, (int)dt, n);
  return hipGetLastError();
}

}  // namespace ttk
