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

// ---------------------------------------------------------------- loads
typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ const TT_GLOBAL_AS T* gptr(const T* p) {
  return (const TT_GLOBAL_AS T*)p;
}

// VEC consecutive elements of X converted to FP32 (streamed: non-temporal).
template <typename T, int VEC>
struct Ld;
template <>
struct Ld<float, 1> {
  static __device__ __forceinline__ void get(const float* p, float* o) { o[0] = __builtin_nontemporal_load(gptr(p)); }
};
template <>
struct Ld<float, 2> {
  static __device__ __forceinline__ void get(const float* p, float* o) {
    const f2 v = __builtin_nontemporal_load(gptr(reinterpret_cast<const f2*>(p)));
    o[0] = v.x;
    o[1] = v.y;
  }
};
template <>
struct Ld<float, 4> {
  static __device__ __forceinline__ void get(const float* p, float* o) {
    const f4 v = __builtin_nontemporal_load(gptr(reinterpret_cast<const f4*>(p)));
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <int VEC>
struct Ld<double, VEC> {
  static __device__ __forceinline__ void get(const double* p, float* o) {
#pragma unroll
    for (int s = 0; s < VEC; ++s) o[s] = (float)__builtin_nontemporal_load(gptr(p + s));
  }
};
template <int VEC>
struct Ld<__hip_bfloat16, VEC> {
  static __device__ __forceinline__ void get(const __hip_bfloat16* p, float* o) {
    const unsigned short* q = reinterpret_cast<const unsigned short*>(p);
#pragma unroll
    for (int s = 0; s < VEC; ++s) o[s] = __uint_as_float(((unsigned)__builtin_nontemporal_load(gptr(q + s))) << 16);
  }
};

// Regular (cached) loads: pass 1's row tiles share the L2 lines where a
// column's segments meet, and the tiles of one chunk run on one XCD.
template <typename T, int VEC>
struct LdC;
template <int VEC>
struct LdC<float, VEC> {
  static __device__ __forceinline__ void get(const float* p, float* o) {
    if constexpr (VEC == 4) {
      const f4 v = *gptr(reinterpret_cast<const f4*>(p));
      o[0] = v.x;
      o[1] = v.y;
      o[2] = v.z;
      o[3] = v.w;
    } else if constexpr (VEC == 2) {
      const f2 v = *gptr(reinterpret_cast<const f2*>(p));
      o[0] = v.x;
      o[1] = v.y;
    } else {
      o[0] = *gptr(p);
    }
  }
};
template <int VEC>
struct LdC<double, VEC> {
  static __device__ __forceinline__ void get(const double* p, float* o) {
#pragma unroll
    for (int s = 0; s < VEC; ++s) o[s] = (float)*gptr(p + s);
  }
};
template <int VEC>
struct LdC<__hip_bfloat16, VEC> {
  static __device__ __forceinline__ void get(const __hip_bfloat16* p, float* o) {
    const unsigned short* q = reinterpret_cast<const unsigned short*>(p);
#pragma unroll
    for (int s = 0; s < VEC; ++s) o[s] = __uint_as_float(((unsigned)*gptr(q + s)) << 16);
  }
};

// Workgroups are dispatched to the 8 XCDs round-robin by linear id.  Pass 1
// maps linear id b to (row tile, chunk) so that every row tile of a chunk
// lands on XCD b % 8: chunk = 8 * (s / tiles) + b % 8, tile = s % tiles with
// s = b / 8.  Returns false for the padding ids of a ragged last group.
__device__ __forceinline__ bool xcd_tile(int b, int tiles, int chunks, int& tile, int& chunk) {
  const int x = b & 7, sidx = b >> 3;
  tile = sidx % tiles;
  chunk = 8 * (sidx / tiles) + x;
  return chunk < chunks;
}

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row of the 32x32 result held by lane `lane`, register v.
__device__ __forceinline__ int mfma_row(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// ------------------------------------------------------------------ pass 1
// Grid of tiles x chunks blocks (XCD-aware order, see xcd_tile), NW waves per
// block.  Block (tp, c) owns
// the row tile [32 VEC tp, 32 VEC (tp+1)) and a contiguous range of column
// pairs, which its waves take round-robin.  Lane i + 32h loads VEC
// consecutive rows p0 + VEC i .. +VEC-1 of column 2q + h with one vector load;
// element s feeds MFMA s, whose 32 result rows are p0 + VEC i' + s.  All VEC
// MFMAs of a step share the right-interface operand B(a, j).  The next
// step's loads are issued before the current step's MFMAs.  The waves' tiles
// are added in LDS in wave order and the block writes one FP32 partial tile;
// k_pass1_reduce adds the chunks' partials in chunk order in FP64.
template <typename T, int VEC, int NW, int NTN>
__global__ void __launch_bounds__(NW * 64) k_pass1(const T* __restrict__ X, int64_t P, int64_t J, int r,
                                                   const float* __restrict__ B, float* __restrict__ part,
                                                   int tiles, int chunks, const PassDesc* __restrict__ batch) {
  if (batch) {  // member blockIdx.y of a batch
    const PassDesc& pp = batch[blockIdx.y];
    X = static_cast<const T*>(pp.x);
    B = pp.w;
    part = pp.ws;
    P = pp.P;
    J = pp.J;
    r = pp.r;
    tiles = pp.tiles;
    chunks = pp.chunks;
  }
  constexpr int TILEF = NTN * VEC * 1024;
  // LDS slots for the wave reduction: waves add into slot w % SLOTS in
  // rounds, in wave order, so the sum is reproducible.
  constexpr int SLOTS = (NW * TILEF <= 16384) ? NW : (16384 / TILEF);
  __shared__ float red[SLOTS * TILEF];
  int tp, c;
  if (!xcd_tile((int)blockIdx.x, tiles, chunks, tp, c)) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t p0 = (int64_t)tp * 32 * VEC;
  const int64_t npairs = (J + 1) >> 1;
  const int64_t pb = npairs * c / chunks, pe = npairs * (c + 1) / chunks;
  const int64_t prow = p0 + (int64_t)VEC * (lane & 31);
  const bool rowok = prow < P;  // P % VEC == 0, so a vector is all in or all out
  const int half = lane >> 5;
  const int acol = lane & 31;
  floatx16 acc[NTN][VEC];
#pragma unroll
  for (int t = 0; t < NTN; ++t)
#pragma unroll
    for (int s = 0; s < VEC; ++s) acc[t][s] = floatx16{0};

  // Column pairs per load batch: the next batch is in flight while the MFMAs
  // of the current one run (two batches stay under 63 outstanding loads).
  constexpr int U = (VEC == 1) ? 8 : 4;
  // Per-lane pointers of this wave's first column pair.  Rows past P (last
  // tile only) read row P - VEC; columns past the chunk read its last column
  // (pointer clamped).  Both are zeroed by masks applied at MFMA time, so the
  // load batches themselves never wait on their data: the next batch stays
  // in flight while the current one is multiplied.
  const int64_t prow_c = rowok ? prow : P - VEC;
  const int64_t j_first = 2 * (pb + w) + half;
  const int64_t jend = (2 * pe < J) ? 2 * pe : J;
  int acol_c[NTN];
#pragma unroll
  for (int t = 0; t < NTN; ++t) {
    const int a = acol + 32 * t;
    acol_c[t] = a < r ? a : r - 1;
  }
  const int64_t xstep = 2 * (int64_t)NW * P;   // one column pair per wave step
  const int64_t bstep = 2 * (int64_t)NW * r;
  const T* xp = X + prow_c + P * j_first;
  const T* xlast = X + prow_c + P * (jend - 1);
  const float* bp = B + (int64_t)r * j_first;
  const float* blast = B + (int64_t)r * (jend - 1);
  const int64_t nsteps = (pe > pb + w) ? (pe - (pb + w) + NW - 1) / NW : 0;

  float xa0[U][VEC], bb0[U][NTN], xa1[U][VEC], bb1[U][NTN];
  // Interface values first (they come from L2), then the slice vectors, so
  // the MFMAs of column pair u wait only for the loads up to pair u.
  auto load = [&](float (&xa)[U][VEC], float (&bb)[U][NTN], int64_t i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float* b = bp + (i0 + u) * bstep;
      b = b < blast ? b : blast;
#pragma unroll
      for (int t = 0; t < NTN; ++t) bb[u][t] = *gptr(b + acol_c[t]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T* x = xp + (i0 + u) * xstep;
      x = x < xlast ? x : xlast;
      LdC<T, VEC>::get(x, xa[u]);
    }
  };
  // Rows past P and ranks past r only reach outputs that are never stored; a
  // column past the chunk is zeroed on the interface operand, so the slice
  // values enter the MFMAs as loaded (no per-element select to wait for).
  auto compute = [&](const float (&xa)[U][VEC], const float (&bb)[U][NTN], int64_t i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool live = j_first + (i0 + u) * 2 * NW < jend;
#pragma unroll
      for (int t = 0; t < NTN; ++t) {
        const float b = live ? bb[u][t] : 0.f;
#pragma unroll
        for (int s = 0; s < VEC; ++s) acc[t][s] = mfma32(xa[u][s], b, acc[t][s]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  // Branch-free steady state: loads past the wave's last step read the
  // clamped column and are masked, so the prefetch is unconditional.
  if (nsteps > 0) {
    // sched_barrier keeps each batch's loads together and ahead of the
    // previous batch's MFMAs (the scheduler would otherwise interleave them).
    load(xa0, bb0, 0);
    for (int64_t i0 = 0; i0 < nsteps; i0 += 2 * U) {
      __builtin_amdgcn_sched_barrier(0);
      load(xa1, bb1, i0 + U);
      __builtin_amdgcn_sched_barrier(0);
      compute(xa0, bb0, i0);
      __builtin_amdgcn_sched_barrier(0);
      load(xa0, bb0, i0 + 2 * U);
      __builtin_amdgcn_sched_barrier(0);
      compute(xa1, bb1, i0 + U);
    }
  }

#pragma unroll
  for (int round = 0; round < NW / SLOTS; ++round) {
    if (w / SLOTS == round) {
      float* slot = red + (w % SLOTS) * TILEF;
#pragma unroll
      for (int t = 0; t < NTN; ++t)
#pragma unroll
        for (int s = 0; s < VEC; ++s)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int e = ((t * VEC + s) * 16 + v) * 64 + lane;
            slot[e] = (round == 0) ? acc[t][s][v] : slot[e] + acc[t][s][v];
          }
    }
    __syncthreads();
  }
  float* out = part + ((int64_t)tp * chunks + c) * TILEF;
  for (int e = threadIdx.x; e < TILEF; e += NW * 64) {
    float sum = 0.f;
#pragma unroll
    for (int ww = 0; ww < SLOTS; ++ww) sum += red[ww * TILEF + e];
    out[e] = sum;
  }
}

// Z(row, col) = sum over chunks of the partial tiles, in FP64.  A block
// covers kRedElems tile elements; its thread (element e, group g) adds the
// chunks g, g + kRedGroups, ... in order, with all of its loads in flight at
// once, and the kRedGroups sums are then added in group order, so the result
// does not depend on the launch (every member of a batch sums the same way).
constexpr int kRedGroups = 4;
constexpr int kRedElems = 256 / kRedGroups;

template <int VEC, int NTN>
__global__ void __launch_bounds__(256) k_pass1_reduce(const float* __restrict__ part, int chunks, int64_t P, int r,
                                                      double* __restrict__ Z, int* __restrict__ flag,
                                                      const PassDesc* __restrict__ batch) {
  if (batch) {
    const PassDesc& pp = batch[blockIdx.y];
    part = pp.ws;
    Z = pp.out;
    flag = pp.flag;
    chunks = pp.chunks;
    P = pp.P;
    r = pp.r;
  }
  constexpr int TILEF = NTN * VEC * 1024;
  __shared__ double red[256];
  const int el = threadIdx.x % kRedElems, g = threadIdx.x / kRedElems;
  const int64_t eg = (int64_t)blockIdx.x * kRedElems + el;
  const int64_t tp = eg / TILEF;
  const int e = (int)(eg % TILEF);
  const int64_t ntiles = (P + 32 * VEC - 1) / (32 * VEC);
  double sum = 0.0;
  if (tp < ntiles) {
    const float* p = part + tp * chunks * TILEF + e;
    for (int c0 = g; c0 < chunks; c0 += 8 * kRedGroups) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int cc = c0 + u * kRedGroups;
        v[u] = cc < chunks ? *gptr(p + (int64_t)cc * TILEF) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += (double)v[u];
    }
  }
  red[threadIdx.x] = sum;
  __syncthreads();
  if (g != 0 || tp >= ntiles) return;
#pragma unroll
  for (int gg = 1; gg < kRedGroups; ++gg) sum += red[gg * kRedElems + el];
  const int t = e / (VEC * 1024), s = (e / 1024) % VEC, v = (e / 64) % 16, ln = e % 64;
  const int64_t row = tp * 32 * VEC + (int64_t)VEC * mfma_row(ln, v) + s;
  const int col = (ln & 31) + 32 * t;
  if (row >= P || col >= r) return;
  Z[row + P * (int64_t)col] = sum;
  if (!isfinite(sum)) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ pass 2
// Grid ceil(J/32) blocks of kPass2Waves waves; block b owns columns [32 b, 32 b + 32)
// and all P rows.  Wave w owns the row slab [w*slab, (w+1)*slab) and stages it
// through its own LDS area in chunks of at most kPass2SlabMax rows, loading
// VEC consecutive rows of a column per lane, so the slice is read in runs
// along its contiguous index.  The MFMA's reduction index k runs over rows:
// lane i + 32g supplies rows kk + 4g + s for the four MFMAs s = 0..3 of a
// step, for both the slice (operand A = X^T) and the left interface
// (operand B).  The waves' tiles are added in LDS in wave order and the
// block writes Y in FP64.  The next chunk's slice loads are held in
// registers while the current chunk's MFMAs run.
constexpr int kLdp = kPass2SlabMax + 4;

template <typename T, int VEC, int NTN>
__global__ void __launch_bounds__(kPass2Waves * 64) k_pass2(const T* __restrict__ X, int64_t P, int64_t J, int r,
                                                            const float* __restrict__ A, double* __restrict__ Y,
                                                            int* __restrict__ flag, int slab, int nchunk,
                                                            const PassDesc* __restrict__ batch) {
  if (batch) {
    const PassDesc& pp = batch[blockIdx.y];
    X = static_cast<const T*>(pp.x);
    A = pp.w;
    Y = pp.out;
    flag = pp.flag;
    P = pp.P;
    J = pp.J;
    r = pp.r;
    slab = (int)(((P + kPass2Waves - 1) / kPass2Waves + 7) & ~7LL);
    nchunk = (slab + kPass2SlabMax - 1) / kPass2SlabMax;
  }
  if ((int64_t)blockIdx.x * 32 >= J) return;  // past this member's columns
  extern __shared__ float lds[];
  constexpr int PER_COL = kPass2SlabMax / VEC;           // vector loads per column and chunk
  constexpr int NLD = (32 * PER_COL + 63) / 64;          // vector loads per lane and chunk
  constexpr int KS = kPass2SlabMax / 8;                  // MFMA k-steps per chunk
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float* Xs = lds + w * 32 * kLdp;
  const int64_t j0 = (int64_t)blockIdx.x * 32;
  const int64_t rb = (int64_t)w * slab;
  const int64_t re = (rb + slab < P) ? rb + slab : P;
  const int g = lane >> 5, jl = lane & 31;
  floatx16 acc[NTN];
#pragma unroll
  for (int t = 0; t < NTN; ++t) acc[t] = floatx16{0};

  auto rows_of = [&](int ch) -> int {
    int64_t rows = re - (rb + (int64_t)ch * kPass2SlabMax);
    if (rows < 0) rows = 0;
    if (rows > kPass2SlabMax) rows = kPass2SlabMax;
    return (int)rows;
  };
  // slice loads of one chunk into registers (lane e -> column e / PER_COL)
  float xr[NLD][VEC];
  // Loads are unconditional (row and column clamped to the slice) so that
  // the wait counts stay exact; out-of-range values are zeroed at the store.
  static_assert((32 * PER_COL) % 64 == 0, "whole vector loads per lane");
  auto load_chunk = [&](int ch) {
    const int64_t c0 = rb + (int64_t)ch * kPass2SlabMax;
#pragma unroll
    for (int it = 0; it < NLD; ++it) {
      const int e = lane + 64 * it;
      const int col = e / PER_COL, row = (e - col * PER_COL) * VEC;
      int64_t p = c0 + row;
      p = p < P - VEC ? p : P - VEC;
      int64_t jj = j0 + col;
      jj = jj < J ? jj : J - 1;
      Ld<T, VEC>::get(X + p + P * jj, xr[it]);
    }
  };
  auto store_chunk = [&](int ch) {
    const int rows = rows_of(ch);
#pragma unroll
    for (int it = 0; it < NLD; ++it) {
      const int e = lane + 64 * it;
      const int col = e / PER_COL, row = (e - col * PER_COL) * VEC;
      const bool colok = j0 + col < J;
      if constexpr (VEC == 4) {  // one 16-byte LDS store (kLdp and row are multiples of 4)
        f4 v;
        v.x = (colok && row + 0 < rows) ? xr[it][0] : 0.f;
        v.y = (colok && row + 1 < rows) ? xr[it][1] : 0.f;
        v.z = (colok && row + 2 < rows) ? xr[it][2] : 0.f;
        v.w = (colok && row + 3 < rows) ? xr[it][3] : 0.f;
        *reinterpret_cast<f4*>(&Xs[col * kLdp + row]) = v;
      } else {
#pragma unroll
        for (int s = 0; s < VEC; ++s) Xs[col * kLdp + row + s] = (colok && row + s < rows) ? xr[it][s] : 0.f;
      }
    }
  };

  if (nchunk > 0) load_chunk(0);
  for (int ch = 0; ch < nchunk; ++ch) {
    const int64_t c0 = rb + (int64_t)ch * kPass2SlabMax;
    const int rows = rows_of(ch);
    const int r8 = (rows + 7) & ~7;
    store_chunk(ch);
    __syncthreads();
    // Interface fragments of every k-step (operand B of k-step k is
    // A(c0 + 8k + 4g + s, a)), issued before the next chunk's slice loads:
    // waits are in issue order, so the MFMAs can then start while the slice
    // prefetch is still in flight.
    float av[KS][NTN][4];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int64_t pbase = c0 + 8 * k + 4 * g;
#pragma unroll
      for (int t = 0; t < NTN; ++t) {
        const int a = jl + 32 * t;
        const int ac = a < r ? a : r - 1;
        if (VEC == 4) {
          const int64_t pc = pbase < P - 3 ? pbase : P - 4;
          const f4 q = *gptr(reinterpret_cast<const f4*>(A + pc + P * (int64_t)ac));
          av[k][t][0] = q.x;
          av[k][t][1] = q.y;
          av[k][t][2] = q.z;
          av[k][t][3] = q.w;
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int64_t p = pbase + s;
            av[k][t][s] = *gptr(A + (p < P ? p : P - 1) + P * (int64_t)ac);
          }
        }
      }
    }
    auto mfma_chunk = [&]() {
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        if (8 * k >= r8) break;
        const float4 xv = *reinterpret_cast<const float4*>(&Xs[jl * kLdp + 8 * k + 4 * g]);
#pragma unroll
        for (int t = 0; t < NTN; ++t) {
          const int a = jl + 32 * t;
          const float am = a < r ? 1.f : 0.f;
          float b[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) b[s] = (8 * k + 4 * g + s < rows) ? av[k][t][s] * am : 0.f;
          acc[t] = mfma32(xv.x, b[0], acc[t]);
          acc[t] = mfma32(xv.y, b[1], acc[t]);
          acc[t] = mfma32(xv.z, b[2], acc[t]);
          acc[t] = mfma32(xv.w, b[3], acc[t]);
        }
      }
    };
    // Separate paths with and without the prefetch keep the wait counts
    // exact on each (a merged path would wait for the prefetch too).
    if (ch + 1 < nchunk) {
      __builtin_amdgcn_sched_barrier(0);
      load_chunk(ch + 1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_chunk();
    } else {
      mfma_chunk();
    }
    __syncthreads();
  }
  // cross-wave reduction in LDS (reuses the staging area), wave order
  int bad = 0;
#pragma unroll
  for (int t = 0; t < NTN; ++t) {
#pragma unroll
    for (int v = 0; v < 16; ++v) lds[(w * 16 + v) * 64 + lane] = acc[t][v];
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += kPass2Waves * 64) {
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


// Pass 2 for FP32 slices with 4 <= P <= 1280 and r <= 32 (the grouped
// kernel).  A block of kPass2gWaves waves owns TPB = NW / NWT
// consecutive 32-column tiles, NWT waves per tile (NWT, a power of two, the
// fewest waves that keep every wave within 2G = 10 eight-row k-steps:
// P <= 80 NWT, so small slices do not spread a few rows over many waves).  The ceil(P/8)
// MFMA k-steps of a tile are split over its waves in contiguous runs (wave i
// of the tile takes steps [K i / NWT, K (i+1) / NWT)), so the waves of a SIMD
// hold about the same number.  A wave issues every load of its rows at once,
// the interface's before the slice's, in 16-row groups: two loads per lane
// cover a group's 32 columns (lane -> column 16h + lane/4, rows 4 (lane%4)
// .. +3, each column read as one 64-byte run; one 16-byte load when
// P % 4 == 0 (V4), else four 4-byte loads).  Group c is then written to two
// 32 x 16 wave-private LDS tiles (slice and interface) and read back as MFMA
// fragments as soon as its loads have landed, so a wave's MFMAs start on its
// first group while the rest of its rows are still in flight; no block
// barrier is needed before the final reduction, which adds each tile's waves
// in order.  Rows past P, columns past J and ranks past r are zeroed at the
// LDS write; groups past the wave's run are loaded (clamped) but not
// multiplied.
constexpr int kPass2gWaves = 16;
constexpr int kPass2gGroups = 5;  // 16-row groups per wave: up to 10 k-steps
constexpr int kPass2gLdp = 20;    // LDS row pitch of a 32 x 16 tile (floats)
constexpr int64_t kPass2gMaxRows = 8LL * 2 * kPass2gGroups * kPass2gWaves;
constexpr size_t kPass2gLds =
    (size_t)kPass2gWaves * 64 * kPass2gLdp * sizeof(float) > (size_t)kPass2gWaves * 1024 * sizeof(float)
        ? (size_t)kPass2gWaves * 64 * kPass2gLdp * sizeof(float)
        : (size_t)kPass2gWaves * 1024 * sizeof(float);

template <int NWT, bool V4>
__global__ void __launch_bounds__(kPass2gWaves * 64) k_pass2g(const float* __restrict__ X, int64_t P, int64_t J, int r,
                                                              const float* __restrict__ A, double* __restrict__ Y,
                                                              int* __restrict__ flag,
                                                              const PassDesc* __restrict__ batch) {
  if (batch) {
    const PassDesc& pp = batch[blockIdx.y];
    X = static_cast<const float*>(pp.x);
    A = pp.w;
    Y = pp.out;
    flag = pp.flag;
    P = pp.P;
    J = pp.J;
    r = pp.r;
  }
  constexpr int NW = kPass2gWaves, TPB = NW / NWT, G = kPass2gGroups, LDP = kPass2gLdp;
  if ((int64_t)blockIdx.x * TPB * 32 >= J) return;  // past this member's columns
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 5, jl = lane & 31;
  const int64_t jb = (int64_t)blockIdx.x * TPB * 32;  // the block's first column
  const int64_t j0 = jb + 32 * (w / NWT);               // this wave's tile
  const int wi = w % NWT;
  const int np = (int)P;  // P <= kPass2gMaxRows
  const int K = (np + 7) >> 3;
  const int kb = K * wi / NWT;
  const int nk = j0 < J ? K * (wi + 1) / NWT - kb : 0;  // a tile past J multiplies nothing
  const int rb = 8 * kb;
  const int lc = lane >> 2, lr = 4 * (lane & 3);
  // four consecutive rows from row p of the column whose first element is
  // base[col] (clamped into the matrix); the 4-byte loads take 32-bit
  // element offsets from the uniform base (P J < 2^30 for this variant)
  auto ld4 = [&](const float* base, int64_t col, int p) -> f4 {
    if constexpr (V4) {
      return *gptr(reinterpret_cast<const f4*>(base + col + (p < np - 4 ? p : np - 4)));
    } else {
      f4 v;
      const unsigned co = (unsigned)col;
#pragma unroll
      for (int s = 0; s < 4; ++s) v[s] = *gptr(base + (co + (unsigned)(p + s < np - 1 ? p + s : np - 1)));
      return v;
    }
  };
  f4 ar[2 * G], xr[2 * G];
#pragma unroll
  for (int c = 0; c < G; ++c)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int a = 16 * h + lc;
      a = a < r ? a : r - 1;
      ar[2 * c + h] = ld4(A, P * (int64_t)a, rb + 16 * c + lr);
    }
#pragma unroll
  for (int c = 0; c < G; ++c)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int64_t jj = j0 + 16 * h + lc;
      jj = jj < J ? jj : J - 1;
      xr[2 * c + h] = ld4(X, P * jj, rb + 16 * c + lr);
    }
  // keep every load ahead of the first LDS write
  __builtin_amdgcn_sched_barrier(0);
  float* Xs = lds + w * 64 * LDP;
  float* As = Xs + 32 * LDP;
  floatx16 acc = floatx16{0};
#pragma unroll
  for (int c = 0; c < G; ++c) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = 16 * h + lc;
      const bool xok = j0 + col < J, aok = col < r;
      f4 v, u;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool rok = rb + 16 * c + lr + s < np;
        v[s] = (xok && rok) ? xr[2 * c + h][s] : 0.f;
        u[s] = (aok && rok) ? ar[2 * c + h][s] : 0.f;
      }
      // the wave's own tiles: its LDS operations complete in order, so the
      // next group's writes cannot overtake this group's reads
      *reinterpret_cast<f4*>(&Xs[col * LDP + lr]) = v;
      *reinterpret_cast<f4*>(&As[col * LDP + lr]) = u;
    }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      if (2 * c + kk < nk) {
        const f4 xv = *reinterpret_cast<const f4*>(&Xs[jl * LDP + 8 * kk + 4 * g]);
        const f4 av = *reinterpret_cast<const f4*>(&As[jl * LDP + 8 * kk + 4 * g]);
        acc = mfma32(xv.x, av.x, acc);
        acc = mfma32(xv.y, av.y, acc);
        acc = mfma32(xv.z, av.z, acc);
        acc = mfma32(xv.w, av.w, acc);
      }
    }
  }
  // reduction in LDS (reuses the tiles): each tile adds its waves in order
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 16; ++v) lds[(w * 16 + v) * 64 + lane] = acc[v];
  __syncthreads();
  int bad = 0;
  for (int e = threadIdx.x; e < TPB * 1024; e += NW * 64) {
    const int t = e >> 10, el = e & 1023;
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NWT; ++q) s += lds[(t * NWT + q) * 1024 + el];
    const int v = el / 64, ln = el % 64;
    const int64_t jj = jb + 32 * t + mfma_row(ln, v);
    const int a = ln & 31;
    if (jj < J && a < r) {
      Y[a + (int64_t)r * jj] = (double)s;
      if (!isfinite(s)) bad = 1;
    }
  }
  if (bad) atomicOr(flag, 1);
}

template <int NWT>
void launch_p2g(hipStream_t st, const float* X, int64_t P, int64_t J, int r, const float* A, double* Y, int* flag,
                const PassLaunch* bl) {
  constexpr int TPB = kPass2gWaves / NWT;
  const unsigned tiles = pass2_grid(J);
  const dim3 grid(bl ? bl->gx : (tiles + TPB - 1) / TPB, bl ? (unsigned)bl->n : 1u);
  const PassDesc* d = bl ? bl->desc : nullptr;
  if (P % 4 == 0)
    hipLaunchKernelGGL((k_pass2g<NWT, true>), grid, dim3(kPass2gWaves * 64), kPass2gLds, st, X, P, J, r, A, Y, flag, d);
  else
    hipLaunchKernelGGL((k_pass2g<NWT, false>), grid, dim3(kPass2gWaves * 64), kPass2gLds, st, X, P, J, r, A, Y, flag,
                       d);
}

template <int NWT>
hipError_t attr2g() {
  hipError_t e = hipFuncSetAttribute((const void*)k_pass2g<NWT, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kPass2gLds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_pass2g<NWT, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kPass2gLds);
  return e;
}

// ------------------------------------------------------------------ launch
template <typename T, int VEC, int NW, int NTN>
hipError_t launch_p1(hipStream_t st, const T* X, int64_t P, int64_t J, int r, const float* B, double* Z, float* ws,
                     int* flag, int chunks, const PassLaunch* bl) {
  const int tiles = (int)((P + 32 * VEC - 1) / (32 * VEC));
  const int groups = (chunks + 7) / 8;
  constexpr int TILEF = NTN * VEC * 1024;
  const int64_t threads = (int64_t)tiles * TILEF;
  const unsigned gx = bl ? bl->gx : (unsigned)(tiles * groups * 8);
  const unsigned grx = bl ? bl->grx : (unsigned)((threads + kRedElems - 1) / kRedElems);
  const unsigned nb = bl ? (unsigned)bl->n : 1u;
  const PassDesc* d = bl ? bl->desc : nullptr;
  const int mask = pass_launch_mask();
  if (mask & 1)
    hipLaunchKernelGGL((k_pass1<T, VEC, NW, NTN>), dim3(gx, nb), dim3(NW * 64), 0, st, X, P, J, r, B, ws, tiles,
                       chunks, d);
  if (hipEvent_t m = pass_mid_event()) {
    const hipError_t e = hipEventRecord(m, st);
    if (e != hipSuccess) return e;
  }
  if (mask & 2)
    hipLaunchKernelGGL((k_pass1_reduce<VEC, NTN>), dim3(grx, nb), dim3(256), 0, st, ws, chunks, P, r, Z, flag, d);
  return hipGetLastError();
}

template <typename T>
hipError_t pass1_t(hipStream_t st, const T* X, const Pass1Plan& pl, int64_t P, int64_t J, int r, const float* B,
                   double* Z, float* ws, int* flag, const PassLaunch* bt) {
  const int c = pl.chunks;
  if (pl.ntn == 1) {
    if (pl.vec == 4) {
      if (pl.waves == 8) return launch_p1<T, 4, 8, 1>(st, X, P, J, r, B, Z, ws, flag, c, bt);
      return launch_p1<T, 4, 4, 1>(st, X, P, J, r, B, Z, ws, flag, c, bt);
    }
    if (pl.vec == 2) {
      if (pl.waves == 8) return launch_p1<T, 2, 8, 1>(st, X, P, J, r, B, Z, ws, flag, c, bt);
      return launch_p1<T, 2, 4, 1>(st, X, P, J, r, B, Z, ws, flag, c, bt);
    }
    if (pl.waves == 16) return launch_p1<T, 1, 16, 1>(st, X, P, J, r, B, Z, ws, flag, c, bt);
    return launch_p1<T, 1, 8, 1>(st, X, P, J, r, B, Z, ws, flag, c, bt);
  }
  if (pl.vec == 2) return launch_p1<T, 2, 4, 2>(st, X, P, J, r, B, Z, ws, flag, c, bt);
  return launch_p1<T, 1, 8, 2>(st, X, P, J, r, B, Z, ws, flag, c, bt);
}

template <typename T, int VEC>
hipError_t pass2_v(hipStream_t st, const T* X, int64_t P, int64_t J, int r, const float* A, double* Y, int* flag,
                   const PassLaunch* bl) {
  int64_t slab = (P + kPass2Waves - 1) / kPass2Waves;
  slab = (slab + 7) & ~7LL;
  const int nchunk = (int)((slab + kPass2SlabMax - 1) / kPass2SlabMax);
  const size_t lds = (size_t)kPass2Waves * 32 * kLdp * sizeof(float);
  const dim3 grid(bl ? bl->gx : pass2_grid(J), bl ? (unsigned)bl->n : 1u);
  const PassDesc* bt = bl ? bl->desc : nullptr;
  const dim3 block(kPass2Waves * 64);
  if (!(pass_launch_mask() & 1))
    ;
  else if (r <= 32)
    hipLaunchKernelGGL((k_pass2<T, VEC, 1>), grid, block, lds, st, X, P, J, r, A, Y, flag, (int)slab, nchunk, bt);
  else
    hipLaunchKernelGGL((k_pass2<T, VEC, 2>), grid, block, lds, st, X, P, J, r, A, Y, flag, (int)slab, nchunk, bt);
  if (hipEvent_t m = pass_mid_event()) {
    const hipError_t e = hipEventRecord(m, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t pass2_t(hipStream_t st, const T* X, int64_t P, int64_t J, int r, const float* A, double* Y, int* flag,
                   const PassLaunch* bl) {
  const int vec = pass2_vec(P);
  if (vec == 4) return pass2_v<T, 4>(st, X, P, J, r, A, Y, flag, bl);
  if (vec == 2) return pass2_v<T, 2>(st, X, P, J, r, A, Y, flag, bl);
  return pass2_v<T, 1>(st, X, P, J, r, A, Y, flag, bl);
}

template <typename T, int VEC, int NTN>
hipError_t attr2(int lds) {
  return hipFuncSetAttribute((const void*)k_pass2<T, VEC, NTN>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

}  // namespace

hipEvent_t& pass_mid_event() {
  thread_local hipEvent_t ev = nullptr;
  return ev;
}

int& pass_launch_mask() {
  thread_local int mask = 3;
  return mask;
}

Pass1Plan pass1_plan(int64_t P, int64_t J, int r, int cus) {
  Pass1Plan pl;
  pl.ntn = r <= 32 ? 1 : 2;
  // Widest row vector that divides P: 128-row tiles (one 512-byte run per
  // column per half-wave) measured fastest on the 1080 x 5760 slice.
  if (pl.ntn == 1) {
    pl.vec = (P % 4 == 0) ? 4 : (P % 2 == 0 ? 2 : 1);
    pl.waves = (pl.vec == 4) ? 8 : (pl.vec == 2 ? 4 : 8);
  } else {
    pl.vec = (P % 2 == 0) ? 2 : 1;
    pl.waves = (pl.vec == 2) ? 4 : 8;
  }
  pl.tiles = (int)((P + 32 * pl.vec - 1) / (32 * pl.vec));
  // about one block per CU, at least 16 column pairs per wave
  const int64_t pairs = (J + 1) / 2;
  int64_t chunks = ((int64_t)cus + pl.tiles - 1) / pl.tiles;
  const int64_t maxc = pairs / (16 * pl.waves);
  if (chunks > maxc) chunks = maxc;
  if (chunks < 1) chunks = 1;
  pl.chunks = (int)chunks;
  return finish_plan(pl, P);
}

Pass1Plan finish_plan(Pass1Plan pl, int64_t P) {
  pl.tiles = (int)((P + 32 * pl.vec - 1) / (32 * pl.vec));
  pl.ws_floats = (size_t)pl.tiles * pl.chunks * pl.ntn * pl.vec * 1024;
  return pl;
}

void pass1_grids(const Pass1Plan& pl, int64_t P, unsigned* gx, unsigned* grx) {
  const int tiles = (int)((P + 32 * pl.vec - 1) / (32 * pl.vec));
  *gx = (unsigned)(tiles * ((pl.chunks + 7) / 8) * 8);
  *grx = (unsigned)(((int64_t)tiles * pl.ntn * pl.vec * 1024 + kRedElems - 1) / kRedElems);
}

unsigned pass2_grid(int64_t J) { return (unsigned)((J + 31) / 32); }
bool pass2_grouped(int64_t P, int64_t J, int r, tt_dtype xdt) {
  if (xdt != TT_F32 || P < 4 || r > 32) return false;
  return P <= kPass2gMaxRows && (P % 4 == 0 || P * J < (1LL << 30));
}
int pass2g_nwt(int64_t P) {
  const int64_t K = (P + 7) / 8;
  int nwt = 1;
  while (nwt < kPass2gWaves && K > 2LL * kPass2gGroups * nwt) nwt *= 2;
  return nwt;
}
int pass2_vec(int64_t P) { return P % 4 == 0 ? 4 : (P % 2 == 0 ? 2 : 1); }

hipError_t pass1(hipStream_t st, const void* X, tt_dtype xdt, const Pass1Plan& pl, int64_t P, int64_t J, int r,
                 const float* B, double* Z, float* ws, int* flag, const PassLaunch* bl) {
  if (r < 1 || r > 64 || (bl && (bl->n < 1 || bl->n > 65535))) return hipErrorInvalidValue;
  switch (xdt) {
    case TT_F32: return pass1_t(st, static_cast<const float*>(X), pl, P, J, r, B, Z, ws, flag, bl);
    case TT_F64: return pass1_t(st, static_cast<const double*>(X), pl, P, J, r, B, Z, ws, flag, bl);
    case TT_BF16: return pass1_t(st, static_cast<const __hip_bfloat16*>(X), pl, P, J, r, B, Z, ws, flag, bl);
  }
  return hipErrorInvalidValue;
}

hipError_t pass2(hipStream_t st, const void* X, tt_dtype xdt, int64_t P, int64_t J, int r, const float* A, double* Y,
                 int* flag, const PassLaunch* bl) {
  if (r < 1 || r > 64 || (bl && (bl->n < 1 || bl->n > 65535))) return hipErrorInvalidValue;
  if (pass2_grouped(P, J, r, xdt)) {
    if (pass_launch_mask() & 1) {
      const float* Xf = static_cast<const float*>(X);
      switch (pass2g_nwt(P)) {
        case 1: launch_p2g<1>(st, Xf, P, J, r, A, Y, flag, bl); break;
        case 2: launch_p2g<2>(st, Xf, P, J, r, A, Y, flag, bl); break;
        case 4: launch_p2g<4>(st, Xf, P, J, r, A, Y, flag, bl); break;
        case 8: launch_p2g<8>(st, Xf, P, J, r, A, Y, flag, bl); break;
        default: launch_p2g<16>(st, Xf, P, J, r, A, Y, flag, bl); break;
      }
    }
    if (hipEvent_t m = pass_mid_event()) {
      const hipError_t e = hipEventRecord(m, st);
      if (e != hipSuccess) return e;
    }
    return hipGetLastError();
  }
  switch (xdt) {
    case TT_F32: return pass2_t(st, static_cast<const float*>(X), P, J, r, A, Y, flag, bl);
    case TT_F64: return pass2_t(st, static_cast<const double*>(X), P, J, r, A, Y, flag, bl);
    case TT_BF16: return pass2_t(st, static_cast<const __hip_bfloat16*>(X), P, J, r, A, Y, flag, bl);
  }
  return hipErrorInvalidValue;
}

hipError_t pass_setup() {
  const int lds = (int)((size_t)kPass2Waves * 32 * kLdp * sizeof(float));
  hipError_t e = hipSuccess;
#define TT_A2(T)                                    \
  if (e == hipSuccess) e = attr2<T, 4, 1>(lds);     \
  if (e == hipSuccess) e = attr2<T, 2, 1>(lds);     \
  if (e == hipSuccess) e = attr2<T, 2, 2>(lds);     \
  if (e == hipSuccess) e = attr2<T, 4, 2>(lds);     \
  if (e == hipSuccess) e = attr2<T, 1, 1>(lds);     \
  if (e == hipSuccess) e = attr2<T, 1, 2>(lds);
  TT_A2(float)
  TT_A2(double)
  TT_A2(__hip_bfloat16)
#undef TT_A2
  if (e == hipSuccess) e = attr2g<1>();
  if (e == hipSuccess) e = attr2g<2>();
  if (e == hipSuccess) e = attr2g<4>();
  if (e == hipSuccess) e = attr2g<8>();
  if (e == hipSuccess) e = attr2g<16>();
  return e;
}

}  // namespace ttk
