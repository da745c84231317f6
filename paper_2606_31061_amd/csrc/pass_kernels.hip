// The two passes of one update that stream the whole slice (FP32 MFMA).
//
// With the split point k* the slice is read as the P x J matrix X = X^<k*>
// (P = I_1..I_k*, J = I_{k*+1}..I_m, p fastest).  Eq. 5's local solves for
// k <= k* all contract X with the right interface B_{k*} first, and those for
// k > k* all contract it with the left interface A_{k*+1} first (Section 4.2
// counts both as the O(I^{n-1} r) term), so one update reads the slice twice:
//   pass 1  Z = X B^T         (P x r, reduction over the long index j)
//   pass 2  Y = A^T X         (r x J, reduction over p)
// Both are tall-skinny and bandwidth-bound.  They use v_mfma_f32_32x32x2_f32:
// operand A element (i, k) in lane i + 32k, operand B element (k, j) in lane
// j + 32k, result (i, j) in lane j + 32*((i/4)%2), register 4*(i/8) + i%4.
#include "tt_internal.h"

namespace ttk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

template <typename T>
__device__ __forceinline__ float ldf(const T* p);
template <>
__device__ __forceinline__ float ldf<float>(const float* p) { return __builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ float ldf<double>(const double* p) { return (float)__builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ float ldf<__hip_bfloat16>(const __hip_bfloat16* p) {
  const unsigned short u = __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p));
  return __uint_as_float(((unsigned)u) << 16);
}

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row of the 32x32 result held by lane `lane`, register v.
__device__ __forceinline__ int mfma_row(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// ------------------------------------------------------------------ pass 1
// Grid (ceil(P/32), chunks); block of WPB waves.  Block (tp, c) owns rows
// [32 tp, 32 tp + 32) and a contiguous range of column pairs; its waves take
// the pairs round-robin.  Each block reduces its waves in LDS, writes one
// partial tile, and the last block of a row tile to finish adds the chunks'
// partials in chunk order (FP64) and writes Z.
template <typename T, int WPB, int NTN>
__global__ void __launch_bounds__(WPB * 64) k_pass1(const T* __restrict__ X, int64_t P, int64_t J, int r,
                                                    const float* __restrict__ B, double* __restrict__ Z,
                                                    float* __restrict__ ws, int* __restrict__ cnt,
                                                    int* __restrict__ flag) {
  __shared__ float red[WPB * NTN * 1024];
  __shared__ int ticket;
  const int tp = blockIdx.x, c = blockIdx.y, chunks = gridDim.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t p0 = (int64_t)tp * 32;
  const int64_t npairs = (J + 1) >> 1;
  const int64_t pb = npairs * c / chunks, pe = npairs * (c + 1) / chunks;
  const int64_t prow = p0 + (lane & 31);
  const bool rowok = prow < P;
  const int half = lane >> 5;
  const int acol = lane & 31;
  floatx16 acc[NTN];
#pragma unroll
  for (int t = 0; t < NTN; ++t) acc[t] = floatx16{0};

  constexpr int U = 8;
  int64_t q = pb + w;
  for (; q + (int64_t)(U - 1) * WPB < pe; q += (int64_t)U * WPB) {
    float xa[U], bb[U][NTN];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = 2 * (q + (int64_t)u * WPB) + half;
      const bool jok = j < J;
      xa[u] = (jok && rowok) ? ldf<T>(X + prow + P * j) : 0.f;
#pragma unroll
      for (int t = 0; t < NTN; ++t) {
        const int a = acol + 32 * t;
        bb[u][t] = (jok && a < r) ? B[a + (int64_t)r * j] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int t = 0; t < NTN; ++t) acc[t] = mfma32(xa[u], bb[u][t], acc[t]);
    }
  }
  for (; q < pe; q += WPB) {
    const int64_t j = 2 * q + half;
    const bool jok = j < J;
    const float xa = (jok && rowok) ? ldf<T>(X + prow + P * j) : 0.f;
#pragma unroll
    for (int t = 0; t < NTN; ++t) {
      const int a = acol + 32 * t;
      const float b = (jok && a < r) ? B[a + (int64_t)r * j] : 0.f;
      acc[t] = mfma32(xa, b, acc[t]);
    }
  }

  // block reduction over waves
#pragma unroll
  for (int t = 0; t < NTN; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) red[((w * NTN + t) * 16 + v) * 64 + lane] = acc[t][v];
  __syncthreads();
  float* part = ws + ((int64_t)tp * chunks + c) * (NTN * 1024);
  for (int e = threadIdx.x; e < NTN * 1024; e += WPB * 64) {
    float s = 0.f;
#pragma unroll
    for (int ww = 0; ww < WPB; ++ww) s += red[ww * NTN * 1024 + e];
    part[e] = s;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) ticket = atomicAdd(&cnt[tp], 1);
  __syncthreads();
  if (ticket != chunks - 1) return;
  __threadfence();
  // last block of this row tile: deterministic sum over chunks
  int bad = 0;
  for (int e = threadIdx.x; e < NTN * 1024; e += WPB * 64) {
    double s = 0.0;
    for (int cc = 0; cc < chunks; ++cc) s += (double)ws[((int64_t)tp * chunks + cc) * (NTN * 1024) + e];
    const int t = e / 1024, v = (e % 1024) / 64, ln = e % 64;
    const int64_t row = p0 + mfma_row(ln, v);
    const int col = (ln & 31) + 32 * t;
    if (row < P && col < r) {
      Z[row + P * (int64_t)col] = s;
      if (!isfinite(s)) bad = 1;
    }
  }
  if (bad) atomicOr(flag, 1);
  if (threadIdx.x == 0) cnt[tp] = 0;
}

// ------------------------------------------------------------------ pass 2
// Grid ceil(J/32) blocks of 16 waves; block b owns columns [32 b, 32 b + 32)
// and all P rows.  Wave w owns the row slab [w*slab, (w+1)*slab) and stages it
// through its own LDS area in chunks of up to kPass2SlabMax rows, so the slice
// is read with consecutive lanes on consecutive rows of a column.  The MFMA's
// reduction index k runs over rows: lane i + 32g supplies rows kk + 4g + s for
// the four MFMAs s = 0..3 of a step, for both the slice (operand A = X^T) and
// the left interface (operand B).  The 16 waves' partial 32x32 tiles are then
// added in LDS in wave order and the block writes Y in FP64.
constexpr int kLdp = kPass2SlabMax + 4;

template <typename T, int NTN>
__global__ void __launch_bounds__(1024) k_pass2(const T* __restrict__ X, int64_t P, int64_t J, int r,
                                                const float* __restrict__ A, double* __restrict__ Y,
                                                int* __restrict__ flag, int slab, int nchunk) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float* Xs = lds + w * 32 * kLdp;
  const int64_t j0 = (int64_t)blockIdx.x * 32;
  const int64_t rb = (int64_t)w * slab;
  const int64_t re = (rb + slab < P) ? rb + slab : P;
  const int g = lane >> 5, jl = lane & 31;
  floatx16 acc[NTN];
#pragma unroll
  for (int t = 0; t < NTN; ++t) acc[t] = floatx16{0};

  for (int ch = 0; ch < nchunk; ++ch) {
    const int64_t c0 = rb + (int64_t)ch * kPass2SlabMax;
    int64_t rows = re - c0;
    if (rows < 0) rows = 0;
    if (rows > kPass2SlabMax) rows = kPass2SlabMax;
    const int r8 = (int)((rows + 7) & ~7LL);
    // stage X(c0 .. c0+r8, j0 .. j0+32) -> Xs[col][row]
    for (int e = lane; e < 32 * r8; e += 64) {
      const int col = e / r8, row = e - col * r8;
      const int64_t jj = j0 + col;
      float v = 0.f;
      if (row < rows && jj < J) v = ldf<T>(X + (c0 + row) + P * jj);
      Xs[col * kLdp + row] = v;
    }
    __syncthreads();
    for (int kk = 0; kk < r8; kk += 8) {
      const float4 xv = *reinterpret_cast<const float4*>(&Xs[jl * kLdp + kk + 4 * g]);
      const int64_t pbase = c0 + kk + 4 * g;
#pragma unroll
      for (int t = 0; t < NTN; ++t) {
        const int a = jl + 32 * t;
        float av[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int64_t p = pbase + s;
          av[s] = (a < r && p < c0 + rows) ? A[p + P * (int64_t)a] : 0.f;
        }
        acc[t] = mfma32(xv.x, av[0], acc[t]);
        acc[t] = mfma32(xv.y, av[1], acc[t]);
        acc[t] = mfma32(xv.z, av[2], acc[t]);
        acc[t] = mfma32(xv.w, av[3], acc[t]);
      }
    }
    __syncthreads();
  }
  // cross-wave reduction in LDS (reuses the staging area)
  int bad = 0;
#pragma unroll
  for (int t = 0; t < NTN; ++t) {
#pragma unroll
    for (int v = 0; v < 16; ++v) lds[(w * 16 + v) * 64 + lane] = acc[t][v];
    __syncthreads();
    {
      const int e = threadIdx.x;  // 1024 entries of the tile
      float s = 0.f;
#pragma unroll
      for (int ww = 0; ww < kPass2Waves; ++ww) s += lds[ww * 1024 + e];
      const int v = e / 64, ln = e % 64;
      const int64_t jj = j0 + mfma_row(ln, v);
      const int a = (ln & 31) + 32 * t;
      if (jj < J && a < r) {
        Y[a + (int64_t)r * jj] = (double)s;
        if (!isfinite(s)) bad = 1;
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(flag, 1);
}

template <typename T>
hipError_t pass1_t(hipStream_t st, const T* X, int64_t P, int64_t J, int r, const float* B, double* Z, float* ws,
                   int* cnt, int* flag, int chunks, int waves) {
  const dim3 grid((unsigned)pass1_tiles(P), (unsigned)chunks);
  if (r <= 32) {
    if (waves == 4) hipLaunchKernelGGL((k_pass1<T, 4, 1>), grid, dim3(256), 0, st, X, P, J, r, B, Z, ws, cnt, flag);
    else hipLaunchKernelGGL((k_pass1<T, 8, 1>), grid, dim3(512), 0, st, X, P, J, r, B, Z, ws, cnt, flag);
  } else {
    hipLaunchKernelGGL((k_pass1<T, 4, 2>), grid, dim3(256), 0, st, X, P, J, r, B, Z, ws, cnt, flag);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t pass2_t(hipStream_t st, const T* X, int64_t P, int64_t J, int r, const float* A, double* Y, int* flag) {
  int64_t slab = (P + kPass2Waves - 1) / kPass2Waves;
  slab = (slab + 7) & ~7LL;
  const int nchunk = (int)((slab + kPass2SlabMax - 1) / kPass2SlabMax);
  const size_t lds = (size_t)kPass2Waves * 32 * kLdp * sizeof(float);
  const dim3 grid((unsigned)((J + 31) / 32));
  if (r <= 32)
    hipLaunchKernelGGL((k_pass2<T, 1>), grid, dim3(1024), lds, st, X, P, J, r, A, Y, flag, (int)slab, nchunk);
  else
    hipLaunchKernelGGL((k_pass2<T, 2>), grid, dim3(1024), lds, st, X, P, J, r, A, Y, flag, (int)slab, nchunk);
  return hipGetLastError();
}

}  // namespace

int pass1_tiles(int64_t P) { return (int)((P + 31) / 32); }

size_t pass1_ws_floats(int64_t P, int r, int chunks) {
  const int ntn = r <= 32 ? 1 : 2;
  return (size_t)pass1_tiles(P) * chunks * ntn * 1024;
}

hipError_t pass1(hipStream_t st, const void* X, tt_dtype xdt, int64_t P, int64_t J, int r, const float* B, double* Z,
                 float* ws, int* cnt, int* flag, int chunks, int waves) {
  if (r < 1 || r > 64) return hipErrorInvalidValue;
  switch (xdt) {
    case TT_F32: return pass1_t(st, static_cast<const float*>(X), P, J, r, B, Z, ws, cnt, flag, chunks, waves);
    case TT_F64: return pass1_t(st, static_cast<const double*>(X), P, J, r, B, Z, ws, cnt, flag, chunks, waves);
    case TT_BF16:
      return pass1_t(st, static_cast<const __hip_bfloat16*>(X), P, J, r, B, Z, ws, cnt, flag, chunks, waves);
  }
  return hipErrorInvalidValue;
}

hipError_t pass2(hipStream_t st, const void* X, tt_dtype xdt, int64_t P, int64_t J, int r, const float* A, double* Y,
                 int* flag) {
  if (r < 1 || r > 64) return hipErrorInvalidValue;
  switch (xdt) {
    case TT_F32: return pass2_t(st, static_cast<const float*>(X), P, J, r, A, Y, flag);
    case TT_F64: return pass2_t(st, static_cast<const double*>(X), P, J, r, A, Y, flag);
    case TT_BF16: return pass2_t(st, static_cast<const __hip_bfloat16*>(X), P, J, r, A, Y, flag);
  }
  return hipErrorInvalidValue;
}

hipError_t pass_setup() {
  const int lds = (int)((size_t)kPass2Waves * 32 * kLdp * sizeof(float));
  hipError_t e;
  e = hipFuncSetAttribute((const void*)k_pass2<float, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_pass2<float, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_pass2<double, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_pass2<double, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_pass2<__hip_bfloat16, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_pass2<__hip_bfloat16, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             lds);
}

}  // namespace ttk
