// BF16-input, FP32-accumulate variants of the two slice passes.
//
// The contractions are those of pass_kernels.hip (pass 1: Z = X B^T, pass 2:
// Y = A^T X, X the P x J unfolding of the slice at the split point, p
// fastest); here both operands are rounded to BF16 (round to nearest even)
// and multiplied with v_mfma_f32_32x32x16_bf16, accumulating in FP32.  The
// MFMA's layout: operand A element (i, k) in lane i + 32 (k / 8), slot k % 8;
// operand B element (k, j) in lane j + 32 (k / 8), slot k % 8; result (i, j)
// in lane j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4.  Any bijection
// between the reduction index and (lane half, slot) gives the same product,
// which is what lets each lane take its operands from contiguous memory.
//
// A block reduces its waves' tiles in LDS in wave order.  When one block
// covers the whole reduction of its tile it writes the FP64 result itself;
// otherwise it stores an FP32 partial tile and a second, small kernel adds the
// tile's partials in FP64 in chunk order.  (A single launch in which the last
// block to arrive finishes the tile needs device-scope release/acquire fences
// in every block; measured here, that version ran many times slower than the
// two launches.)  The sums never depend on block timing.
#include "tt_internal.h"

namespace ttk {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to BF16 and packed (lo in bits 0..15).
__device__ __forceinline__ unsigned pk(float lo, float hi) {
  const float2v f = {lo, hi};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f, bf16x2));
}

__device__ __forceinline__ floatx16 mfma_bf16(u32x4 a, u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

// Row of the 32x32 result held by lane `lane`, register v.
__device__ __forceinline__ int res_row(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// VEC consecutive slice elements as packed BF16 pairs (element 2d in the low
// half of word d; VEC = 1: the element in the low half of word 0).
template <typename T, int VEC>
struct LdB;
template <int VEC>
struct LdB<__hip_bfloat16, VEC> {
  static constexpr int W = VEC >= 2 ? VEC / 2 : 1;
  static __device__ __forceinline__ void get(const __hip_bfloat16* p, unsigned* o) {
    if constexpr (VEC == 8) {
      const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
      o[0] = v.x;
      o[1] = v.y;
      o[2] = v.z;
      o[3] = v.w;
    } else if constexpr (VEC == 4) {
      const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
      o[0] = v.x;
      o[1] = v.y;
    } else if constexpr (VEC == 2) {
      o[0] = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p));
    } else {
      o[0] = __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p));
    }
  }
};
template <int VEC>
struct LdB<float, VEC> {
  static constexpr int W = VEC >= 2 ? VEC / 2 : 1;
  static __device__ __forceinline__ void get(const float* p, unsigned* o) {
    if constexpr (VEC >= 4) {
      typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int h = 0; h < VEC / 4; ++h) {
        const f4 v = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p) + h);
        o[2 * h] = pk(v.x, v.y);
        o[2 * h + 1] = pk(v.z, v.w);
      }
    } else if constexpr (VEC == 2) {
      const float2v v = __builtin_nontemporal_load(reinterpret_cast<const float2v*>(p));
      o[0] = pk(v.x, v.y);
    } else {
      o[0] = pk(__builtin_nontemporal_load(p), 0.f);
    }
  }
};
template <int VEC>
struct LdB<double, VEC> {
  static constexpr int W = VEC >= 2 ? VEC / 2 : 1;
  static __device__ __forceinline__ void get(const double* p, unsigned* o) {
    if constexpr (VEC >= 2) {
#pragma unroll
      for (int d = 0; d < VEC / 2; ++d)
        o[d] = pk((float)__builtin_nontemporal_load(p + 2 * d), (float)__builtin_nontemporal_load(p + 2 * d + 1));
    } else {
      o[0] = pk((float)__builtin_nontemporal_load(p), 0.f);
    }
  }
};

// Workgroups are dispatched to the 8 XCDs round-robin by linear id; every row
// tile of one chunk runs on XCD b % 8 (as in pass_kernels.hip).
__device__ __forceinline__ bool xcd_tile_b(int b, int tiles, int chunks, int& tile, int& chunk) {
  const int x = b & 7, sidx = b >> 3;
  tile = sidx % tiles;
  chunk = 8 * (sidx / tiles) + x;
  return chunk < chunks;
}

// Wave partial tiles into LDS: waves add into slot w % SLOTS in rounds, in
// wave order.  Ends with a barrier.
template <int NW, int SLOTS, int TILEF, class Get>
__device__ __forceinline__ void waves_to_lds(float* red, int w, int lane, Get get) {
#pragma unroll
  for (int round = 0; round < NW / SLOTS; ++round) {
    if (w / SLOTS == round) {
      float* slot = red + (w % SLOTS) * TILEF;
#pragma unroll
      for (int k = 0; k < TILEF / 64; ++k) {
        const int e = k * 64 + lane;
        slot[e] = (round == 0) ? get(k) : slot[e] + get(k);
      }
    }
    __syncthreads();
  }
}

// With one chunk the block finishes its own tile (returns true); otherwise it
// stores its partial tile (the slot sums) for the reduction kernel.
template <int NT, int SLOTS, int TILEF>
__device__ __forceinline__ bool finish_here(const float* red, float* part_tile, int chunks) {
  if (chunks == 1) return true;
  for (int e = threadIdx.x; e < TILEF; e += NT) {
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < SLOTS; ++w) s += red[w * TILEF + e];
    part_tile[e] = s;
  }
  return false;
}

// Element e of a tile finished in its block: the slot sums.
template <int SLOTS, int TILEF>
__device__ __forceinline__ double slot_sum(const float* red, int e) {
  float s = 0.f;
#pragma unroll
  for (int w = 0; w < SLOTS; ++w) s += red[w * TILEF + e];
  return (double)s;
}

// LDS floats for the wave reduction (static LDS stays under 64 KB).
constexpr int kRedFloats = 16000;
// Waves per block: the widest tiles hold about 400 registers per lane, so one
// wave per SIMD.
constexpr int kWavesB = 4;

// LDS slots of the wave reduction: a divisor of the wave count (a power of
// two) whose slots fit in kRedFloats.
constexpr int slots_for(int nw, int tilef) {
  int s = nw;
  while (s > 1 && s * tilef > kRedFloats) s /= 2;
  return s;
}

// ------------------------------------------------------------------ pass 1
// Block (tp, c): rows [32 VEC tp, 32 VEC (tp + 1)), column groups (16 columns
// each) [gb, ge) of chunk c, taken round-robin by the NW waves.  For group q
// lane i + 32h loads, for e = 0..7, the VEC rows 32 VEC tp + VEC i .. of
// column 16 q + 8 h + e in one vector; MFMA s (s < VEC) takes row
// 32 VEC tp + VEC i + s with reduction slot e <-> column 16 q + 8 h + e, so
// the VEC MFMAs of a step share the interface operand.  Rows past P read the
// last rows again (their results are not stored); columns past J are clamped
// and their interface values zeroed.
template <typename T, int VEC, int NW, int NTN>
__global__ void __launch_bounds__(NW * 64) k_pass1b(const T* __restrict__ X, int64_t P, int64_t J, int r,
                                                    const float* __restrict__ B, float* __restrict__ ws,
                                                    double* __restrict__ Z, int* __restrict__ flag, int tiles,
                                                    int chunks, const PassDesc* __restrict__ batch) {
  if (batch) {
    const PassDesc& pp = batch[blockIdx.y];
    X = static_cast<const T*>(pp.x);
    B = pp.w;
    ws = pp.ws;
    Z = pp.out;
    flag = pp.flag;
    P = pp.P;
    J = pp.J;
    r = pp.r;
    tiles = pp.tiles;
    chunks = pp.chunks;
  }
  constexpr int TILEF = NTN * VEC * 1024;
  constexpr int SLOTS = slots_for(NW, TILEF);
  static_assert(NW % SLOTS == 0 && SLOTS * TILEF <= kRedFloats, "wave reduction slots");
  constexpr int WD = LdB<T, VEC>::W;
  __shared__ float red[SLOTS * TILEF];
  int tp, c;
  if (!xcd_tile_b((int)blockIdx.x, tiles, chunks, tp, c)) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 31, h = lane >> 5;
  const int64_t p0 = (int64_t)tp * 32 * VEC;
  int64_t prow = p0 + (int64_t)VEC * li;
  if (prow > P - VEC) prow = P - VEC;
  const int64_t ngr = (J + 15) >> 4;
  const int64_t gb = ngr * c / chunks, ge = ngr * (c + 1) / chunks;
  int acol[NTN];
  float amask[NTN];
#pragma unroll
  for (int t = 0; t < NTN; ++t) {
    const int a = li + 32 * t;
    acol[t] = a < r ? a : r - 1;
    amask[t] = a < r ? 1.f : 0.f;
  }
  floatx16 acc[NTN][VEC];
#pragma unroll
  for (int t = 0; t < NTN; ++t)
#pragma unroll
    for (int s = 0; s < VEC; ++s) acc[t][s] = floatx16{0};

  const int64_t nst = (ge > gb + w) ? (ge - gb - w + NW - 1) / NW : 0;
  auto group = [&](int64_t st) -> int64_t {
    const int64_t q = gb + w + st * NW;
    return q < ge ? q : ge - 1;
  };
  unsigned xa0[8][WD], xa1[8][WD];
  float bv0[NTN][8], bv1[NTN][8];
  auto load = [&](unsigned (&xd)[8][WD], float (&bv)[NTN][8], int64_t q) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int64_t j = 16 * q + 8 * h + e;
      j = j < J ? j : J - 1;
      LdB<T, VEC>::get(X + prow + P * j, xd[e]);
#pragma unroll
      for (int t = 0; t < NTN; ++t) bv[t][e] = B[acol[t] + (int64_t)r * j];
    }
  };
  auto compute = [&](const unsigned (&xd)[8][WD], const float (&bv)[NTN][8], int64_t q) {
    u32x4 bo[NTN];
#pragma unroll
    for (int t = 0; t < NTN; ++t) {
      float m[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) m[e] = (16 * q + 8 * h + e < J) ? bv[t][e] * amask[t] : 0.f;
      bo[t] = u32x4{pk(m[0], m[1]), pk(m[2], m[3]), pk(m[4], m[5]), pk(m[6], m[7])};
    }
#pragma unroll
    for (int s = 0; s < VEC; ++s) {
      const unsigned sel = (s & 1) ? 0x07060302u : 0x05040100u;
      const int d = VEC >= 2 ? s >> 1 : 0;
      const u32x4 a = {__builtin_amdgcn_perm(xd[1][d], xd[0][d], sel), __builtin_amdgcn_perm(xd[3][d], xd[2][d], sel),
                       __builtin_amdgcn_perm(xd[5][d], xd[4][d], sel), __builtin_amdgcn_perm(xd[7][d], xd[6][d], sel)};
#pragma unroll
      for (int t = 0; t < NTN; ++t) acc[t][s] = mfma_bf16(a, bo[t], acc[t][s]);
    }
  };
  if (nst > 0) {
    load(xa0, bv0, group(0));
    for (int64_t st = 0; st < nst; st += 2) {
      __builtin_amdgcn_sched_barrier(0);
      load(xa1, bv1, group(st + 1));
      __builtin_amdgcn_sched_barrier(0);
      compute(xa0, bv0, group(st));
      if (st + 1 < nst) {
        __builtin_amdgcn_sched_barrier(0);
        load(xa0, bv0, group(st + 2));
        __builtin_amdgcn_sched_barrier(0);
        compute(xa1, bv1, group(st + 1));
      }
    }
  }

  waves_to_lds<NW, SLOTS, TILEF>(red, w, lane, [&](int k) { return acc[k / (VEC * 16)][(k / 16) % VEC][k % 16]; });
  if (!finish_here<NW * 64, SLOTS, TILEF>(red, ws + ((int64_t)tp * chunks + c) * TILEF, chunks)) return;
  int bad = 0;
  for (int e = threadIdx.x; e < TILEF; e += NW * 64) {
    const int t = e / (VEC * 1024), s = (e / 1024) % VEC, v = (e / 64) % 16, ln = e % 64;
    const int64_t row = p0 + (int64_t)VEC * res_row(ln, v) + s;
    const int col = (ln & 31) + 32 * t;
    if (row >= P || col >= r) continue;
    const double sum = slot_sum<SLOTS, TILEF>(red, e);
    Z[row + P * (int64_t)col] = sum;
    if (!isfinite(sum)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ pass 2
// Block (ct, rc): columns [32 ct, 32 ct + 32) and the row superblocks (64
// rows each) [sb, se) of row chunk rc, taken round-robin by the NW waves.  In
// superblock u, lane i + 32h loads rows 64 u + 32 h .. + 31 of column
// 32 ct + i as four 8-row vectors; MFMA q (q < 4) takes reduction slot e <->
// row 64 u + 32 h + 8 q + e for both operands (slice and left interface).
// Columns past J are clamped (their results are not stored); rows past P get
// zero interface values.  VX: P % 8 == 0, so an 8-row vector is wholly inside
// or wholly past the slice; otherwise rows are loaded one by one.
template <typename T, int NW, int NTN, bool VX>
__global__ void __launch_bounds__(NW * 64) k_pass2b(const T* __restrict__ X, int64_t P, int64_t J, int r,
                                                    const float* __restrict__ A, float* __restrict__ ws,
                                                    double* __restrict__ Y, int* __restrict__ flag, int ctiles,
                                                    int rchunks, const PassDesc* __restrict__ batch) {
  if (batch) {
    const PassDesc& pp = batch[blockIdx.y];
    X = static_cast<const T*>(pp.x);
    A = pp.w;
    ws = pp.ws;
    Y = pp.out;
    flag = pp.flag;
    P = pp.P;
    J = pp.J;
    r = pp.r;
    ctiles = pp.tiles;
    rchunks = pp.chunks;
  }
  constexpr int TILEF = NTN * 1024;
  constexpr int SLOTS = slots_for(NW, TILEF);
  static_assert(NW % SLOTS == 0 && SLOTS * TILEF <= kRedFloats, "wave reduction slots");
  __shared__ float red[SLOTS * TILEF];
  // no XCD grouping: every slice element is read once, and the left
  // interface is small enough to stay in every XCD's L2
  const int ct = (int)blockIdx.x / rchunks, rc = (int)blockIdx.x % rchunks;
  if (ct >= ctiles) return;  // past this member's columns
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 31, h = lane >> 5;
  int64_t jc = (int64_t)ct * 32 + li;
  jc = jc < J ? jc : J - 1;
  const T* xcol = X + P * jc;
  const int64_t nsb = (P + 63) >> 6;
  const int64_t sb = nsb * rc / rchunks, se = nsb * (rc + 1) / rchunks;
  const int64_t nst = (se > sb + w) ? (se - sb - w + NW - 1) / NW : 0;
  const float* acolp[NTN];
  float amask[NTN];
#pragma unroll
  for (int t = 0; t < NTN; ++t) {
    const int a = li + 32 * t;
    acolp[t] = A + P * (int64_t)(a < r ? a : r - 1);
    amask[t] = a < r ? 1.f : 0.f;
  }
  floatx16 acc[NTN];
#pragma unroll
  for (int t = 0; t < NTN; ++t) acc[t] = floatx16{0};

  auto superblock = [&](int64_t st) -> int64_t {
    const int64_t u = sb + w + st * NW;
    return u < se ? u : se - 1;
  };
  // slice words (4 vectors x 4 packed pairs) and interface values (4 x 8)
  unsigned xw0[4][4], xw1[4][4];
  float av0[NTN][4][8], av1[NTN][4][8];
  auto load = [&](unsigned (&xw)[4][4], float (&av)[NTN][4][8], int64_t u) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t p8 = 64 * u + 32 * h + 8 * q;
      if constexpr (VX) {
        const int64_t pc = p8 < P ? p8 : P - 8;
        LdB<T, 8>::get(xcol + pc, xw[q]);
#pragma unroll
        for (int t = 0; t < NTN; ++t) {
          const float4 a0 = *reinterpret_cast<const float4*>(acolp[t] + pc);
          const float4 a1 = *reinterpret_cast<const float4*>(acolp[t] + pc + 4);
          av[t][q][0] = a0.x;
          av[t][q][1] = a0.y;
          av[t][q][2] = a0.z;
          av[t][q][3] = a0.w;
          av[t][q][4] = a1.x;
          av[t][q][5] = a1.y;
          av[t][q][6] = a1.z;
          av[t][q][7] = a1.w;
        }
      } else {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          unsigned lo, hi;
          int64_t pa = p8 + 2 * d, pb2 = p8 + 2 * d + 1;
          pa = pa < P ? pa : P - 1;
          pb2 = pb2 < P ? pb2 : P - 1;
          LdB<T, 1>::get(xcol + pa, &lo);
          LdB<T, 1>::get(xcol + pb2, &hi);
          xw[q][d] = (lo & 0xffffu) | (hi << 16);
#pragma unroll
          for (int t = 0; t < NTN; ++t) {
            av[t][q][2 * d] = acolp[t][pa];
            av[t][q][2 * d + 1] = acolp[t][pb2];
          }
        }
      }
    }
  };
  auto compute = [&](const unsigned (&xw)[4][4], const float (&av)[NTN][4][8], int64_t u) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t p8 = 64 * u + 32 * h + 8 * q;
      const u32x4 a = {xw[q][0], xw[q][1], xw[q][2], xw[q][3]};
#pragma unroll
      for (int t = 0; t < NTN; ++t) {
        float m[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) m[e] = (p8 + e < P) ? av[t][q][e] * amask[t] : 0.f;
        const u32x4 b = {pk(m[0], m[1]), pk(m[2], m[3]), pk(m[4], m[5]), pk(m[6], m[7])};
        acc[t] = mfma_bf16(a, b, acc[t]);
      }
    }
  };
  if (nst > 0) {
    load(xw0, av0, superblock(0));
    for (int64_t st = 0; st < nst; st += 2) {
      __builtin_amdgcn_sched_barrier(0);
      load(xw1, av1, superblock(st + 1));
      __builtin_amdgcn_sched_barrier(0);
      compute(xw0, av0, superblock(st));
      if (st + 1 < nst) {
        __builtin_amdgcn_sched_barrier(0);
        load(xw0, av0, superblock(st + 2));
        __builtin_amdgcn_sched_barrier(0);
        compute(xw1, av1, superblock(st + 1));
      }
    }
  }

  waves_to_lds<NW, SLOTS, TILEF>(red, w, lane, [&](int k) { return acc[k / 16][k % 16]; });
  if (!finish_here<NW * 64, SLOTS, TILEF>(red, ws + ((int64_t)ct * rchunks + rc) * TILEF, rchunks)) return;
  int bad = 0;
  for (int e = threadIdx.x; e < TILEF; e += NW * 64) {
    const int t = e / 1024, v = (e / 64) % 16, ln = e % 64;
    const int64_t j = (int64_t)ct * 32 + res_row(ln, v);
    const int a = (ln & 31) + 32 * t;
    if (j >= J || a >= r) continue;
    const double sum = slot_sum<SLOTS, TILEF>(red, e);
    Y[a + (int64_t)r * j] = sum;
    if (!isfinite(sum)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}


// ------------------------------------------------------------------ pass 2, staged
// The slice goes through LDS as in pass_kernels.hip's pass 2, here as BF16
// (P % 8 == 0): block b owns columns [32 b, 32 b + 32) and all P rows; wave w
// owns the row slab [w slab, (w + 1) slab) (slab a multiple of 16) and stages
// it in chunks of at most kP2sRows rows, each lane loading 8 consecutive rows
// of a column (16 bytes), so the slice is read in runs along its contiguous
// index.  MFMA step kk takes reduction slot e of lane half g as row
// 16 kk + 8 g + e of the chunk for both operands: the slice from LDS in one
// 16-byte read per lane, the left interface from global memory (two 16-byte
// loads) rounded to BF16.  Rows past the slab are zero in LDS and in the
// interface operand.  The waves' tiles are added in LDS in wave order and the
// block writes Y in FP64; the next chunk's slice loads are held in registers
// while the current chunk's MFMAs run.  Compared with k_pass2b (direct loads,
// 32-byte runs per column) the staging turns the slice reads into 288-byte
// runs.
constexpr int kP2sWaves = 8;
constexpr int kP2sRows = 144;                // rows per chunk, a multiple of 16
constexpr int kP2sLdw = (kP2sRows + 8) / 2;  // LDS words per staged column (a multiple of 4)
constexpr size_t kP2sLds = (size_t)kP2sWaves * 32 * kP2sLdw * sizeof(unsigned);

template <typename T, int NTN>
__global__ void __launch_bounds__(kP2sWaves * 64) k_pass2s(const T* __restrict__ X, int64_t P, int64_t J, int r,
                                                           const float* __restrict__ A, double* __restrict__ Y,
                                                           int* __restrict__ flag, const PassDesc* __restrict__ batch) {
  if (batch) {
    const PassDesc& pp = batch[blockIdx.y];
    X = static_cast<const T*>(pp.x);
    A = pp.w;
    Y = pp.out;
    flag = pp.flag;
    P = pp.P;
    J = pp.J;
    r = pp.r;
  }
  if ((int64_t)blockIdx.x * 32 >= J) return;  // past this member's columns
  extern __shared__ unsigned s2w[];
  constexpr int PER_COL = kP2sRows / 8;   // vector loads per column and chunk
  constexpr int NLD = 32 * PER_COL / 64;  // vector loads per lane and chunk
  constexpr int KS = kP2sRows / 16;       // MFMA steps per chunk
  static_assert((32 * PER_COL) % 64 == 0 && kP2sRows % 16 == 0 && kP2sLdw % 4 == 0, "staging shape");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 5, jl = lane & 31;
  unsigned* Xs = s2w + w * 32 * kP2sLdw;
  const int64_t slab = ((P + kP2sWaves - 1) / kP2sWaves + 15) & ~15LL;
  const int nchunk = (int)((slab + kP2sRows - 1) / kP2sRows);
  const int64_t j0 = (int64_t)blockIdx.x * 32;
  const int64_t rb = (int64_t)w * slab;
  const int64_t re = (rb + slab < P) ? rb + slab : P;
  auto rows_of = [&](int ch) -> int {  // a multiple of 8 (P % 8 == 0)
    int64_t rows = re - (rb + (int64_t)ch * kP2sRows);
    if (rows < 0) rows = 0;
    if (rows > kP2sRows) rows = kP2sRows;
    return (int)rows;
  };
  // Loads are unconditional (row and column clamped to the slice) so that
  // the wait counts stay exact; out-of-range vectors are zeroed at the store.
  unsigned xr[NLD][4];
  auto load_chunk = [&](int ch) {
    const int64_t c0 = rb + (int64_t)ch * kP2sRows;
#pragma unroll
    for (int it = 0; it < NLD; ++it) {
      const int e = lane + 64 * it;
      const int col = e / PER_COL, rv = e - col * PER_COL;
      int64_t p = c0 + 8 * rv;
      p = p < P - 8 ? p : P - 8;
      int64_t jj = j0 + col;
      jj = jj < J ? jj : J - 1;
      LdB<T, 8>::get(X + p + P * jj, xr[it]);
    }
  };
  auto store_chunk = [&](int ch) {
    const int rows = rows_of(ch);
#pragma unroll
    for (int it = 0; it < NLD; ++it) {
      const int e = lane + 64 * it;
      const int col = e / PER_COL, rv = e - col * PER_COL;
      const bool ok = j0 + col < J && 8 * rv < rows;
      const u32x4 v = {ok ? xr[it][0] : 0u, ok ? xr[it][1] : 0u, ok ? xr[it][2] : 0u, ok ? xr[it][3] : 0u};
      *reinterpret_cast<u32x4*>(&Xs[col * kP2sLdw + 4 * rv]) = v;
    }
  };
  floatx16 acc[NTN];
#pragma unroll
  for (int t = 0; t < NTN; ++t) acc[t] = floatx16{0};

  if (nchunk > 0) load_chunk(0);
  for (int ch = 0; ch < nchunk; ++ch) {
    const int64_t c0 = rb + (int64_t)ch * kP2sRows;
    const int rows = rows_of(ch);
    const int r16 = (rows + 15) & ~15;
    store_chunk(ch);
    __syncthreads();
    // interface fragments of every step, issued before the next chunk's
    // slice loads (waits are in issue order)
    u32x4 bv[KS][NTN];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const bool ok = 16 * kk + 8 * g < rows;
      int64_t p = c0 + 16 * kk + 8 * g;
      p = p < P - 8 ? p : P - 8;
#pragma unroll
      for (int t = 0; t < NTN; ++t) {
        const int a = jl + 32 * t;
        const float* ap = A + p + P * (int64_t)(a < r ? a : r - 1);
        const float4 a0 = *reinterpret_cast<const float4*>(ap);
        const float4 a1 = *reinterpret_cast<const float4*>(ap + 4);
        bv[kk][t] = ok ? u32x4{pk(a0.x, a0.y), pk(a0.z, a0.w), pk(a1.x, a1.y), pk(a1.z, a1.w)}
                       : u32x4{0u, 0u, 0u, 0u};
      }
    }
    auto mfma_chunk = [&]() {
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        if (16 * kk >= r16) break;
        const u32x4 xa = *reinterpret_cast<const u32x4*>(&Xs[jl * kP2sLdw + 8 * kk + 4 * g]);
#pragma unroll
        for (int t = 0; t < NTN; ++t) acc[t] = mfma_bf16(xa, bv[kk][t], acc[t]);
      }
    };
    // separate paths with and without the prefetch keep the wait counts exact
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
  float* red = reinterpret_cast<float*>(s2w);
  int bad = 0;
#pragma unroll
  for (int t = 0; t < NTN; ++t) {
#pragma unroll
    for (int v = 0; v < 16; ++v) red[(w * 16 + v) * 64 + lane] = acc[t][v];
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += kP2sWaves * 64) {
      float sum = 0.f;
#pragma unroll
      for (int ww = 0; ww < kP2sWaves; ++ww) sum += red[ww * 1024 + e];
      const int v = e / 64, ln = e % 64;
      const int64_t jj = j0 + res_row(ln, v);
      const int a = (ln & 31) + 32 * t;
      if (jj < J && a < r) {
        Y[a + (int64_t)r * jj] = (double)sum;
        if (!isfinite(sum)) bad = 1;
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ reduce
// out = sum over chunks (in chunk order, FP64) of the partial tiles; thread g
// takes element g % TILEF of tile g / TILEF.  PASS 1: tile = row tile (rows
// 32 VEC tile + VEC res_row + s), out = Z (P x r); PASS 2: tile = column tile,
// out = Y (r x J).
template <int PASS, int VEC, int NTN>
__global__ void __launch_bounds__(256) k_reduceb(const float* __restrict__ ws, int tiles, int chunks, int64_t P,
                                                 int64_t J, int r, double* __restrict__ out,
                                                 int* __restrict__ flag, const PassDesc* __restrict__ batch) {
  if (batch) {
    const PassDesc& pp = batch[blockIdx.y];
    ws = pp.ws;
    out = pp.out;
    flag = pp.flag;
    tiles = pp.tiles;
    chunks = pp.chunks;
    P = pp.P;
    J = pp.J;
    r = pp.r;
  }
  if (chunks == 1) return;  // finished by the pass kernel
  constexpr int TILEF = NTN * VEC * 1024;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t tile = g / TILEF;
  if (tile >= tiles) return;
  const int e = (int)(g % TILEF);
  const int t = e / (VEC * 1024), s = (e / 1024) % VEC, v = (e / 64) % 16, ln = e % 64;
  const int col = (ln & 31) + 32 * t;
  int64_t idx;
  if (PASS == 1) {
    const int64_t row = tile * 32 * VEC + (int64_t)VEC * res_row(ln, v) + s;
    if (row >= P || col >= r) return;
    idx = row + P * (int64_t)col;
  } else {
    const int64_t j = tile * 32 + res_row(ln, v);
    if (j >= J || col >= r) return;
    idx = col + (int64_t)r * j;
  }
  const float* p = ws + tile * chunks * TILEF + e;
  double sum = 0.0;
  int cc = 0;
  for (; cc + 8 <= chunks; cc += 8) {  // eight loads in flight, added in chunk order
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = p[(int64_t)(cc + u) * TILEF];
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += (double)x[u];
  }
  for (; cc < chunks; ++cc) sum += (double)p[(int64_t)cc * TILEF];
  out[idx] = sum;
  if (!isfinite(sum)) atomicOr(flag, 1);
}

template <int PASS, int VEC, int NTN>
hipError_t launch_reduce(hipStream_t st, const PassBPlan& pl, int64_t P, int64_t J, int r, double* out,
                         const void* ws, int* flag, const PassLaunch* bl) {
  if (!(pass_launch_mask() & 2)) return hipSuccess;
  if (!bl && pl.chunks == 1) return hipSuccess;
  if (bl && bl->grx == 0) return hipSuccess;  // no member splits its reduction
  constexpr int TILEF = NTN * VEC * 1024;
  const int64_t threads = (int64_t)pl.tiles * TILEF;
  const unsigned grx = bl ? bl->grx : (unsigned)((threads + 255) / 256);
  hipLaunchKernelGGL((k_reduceb<PASS, VEC, NTN>), dim3(grx, bl ? (unsigned)bl->n : 1u), dim3(256), 0, st,
                     static_cast<const float*>(ws), pl.tiles, pl.chunks, P, J, r, out, flag, bl ? bl->desc : nullptr);
  return hipGetLastError();
}

// ------------------------------------------------------------------ launch
template <typename T, int VEC, int NW, int NTN>
hipError_t launch_p1b(hipStream_t st, const T* X, const PassBPlan& pl, int64_t P, int64_t J, int r, const float* B,
                      double* Z, void* ws, int* flag, const PassLaunch* bl) {
  unsigned gx, grx;
  pass1b_grids(pl, &gx, &grx);
  if (bl) gx = bl->gx;
  if (pass_launch_mask() & 1)
    hipLaunchKernelGGL((k_pass1b<T, VEC, NW, NTN>), dim3(gx, bl ? (unsigned)bl->n : 1u), dim3(NW * 64), 0, st, X, P,
                       J, r, B, static_cast<float*>(ws), Z, flag, pl.tiles, pl.chunks, bl ? bl->desc : nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (hipEvent_t m = pass_mid_event()) e = hipEventRecord(m, st);
  if (e != hipSuccess) return e;
  return launch_reduce<1, VEC, NTN>(st, pl, P, J, r, Z, ws, flag, bl);
}

template <typename T, int NW>
hipError_t p1b_vec(hipStream_t st, const T* X, const PassBPlan& pl, int64_t P, int64_t J, int r, const float* B,
                   double* Z, void* ws, int* flag, const PassLaunch* bt) {
  if (pl.ntn == 1) {
    if (pl.vec == 8) return launch_p1b<T, 8, NW, 1>(st, X, pl, P, J, r, B, Z, ws, flag, bt);
    if (pl.vec == 4) return launch_p1b<T, 4, NW, 1>(st, X, pl, P, J, r, B, Z, ws, flag, bt);
    if (pl.vec == 2) return launch_p1b<T, 2, NW, 1>(st, X, pl, P, J, r, B, Z, ws, flag, bt);
    return launch_p1b<T, 1, NW, 1>(st, X, pl, P, J, r, B, Z, ws, flag, bt);
  }
  if (pl.vec == 4) return launch_p1b<T, 4, NW, 2>(st, X, pl, P, J, r, B, Z, ws, flag, bt);
  if (pl.vec == 2) return launch_p1b<T, 2, NW, 2>(st, X, pl, P, J, r, B, Z, ws, flag, bt);
  return launch_p1b<T, 1, NW, 2>(st, X, pl, P, J, r, B, Z, ws, flag, bt);
}

template <typename T>
hipError_t p1b_t(hipStream_t st, const T* X, const PassBPlan& pl, int64_t P, int64_t J, int r, const float* B,
                 double* Z, void* ws, int* flag, const PassLaunch* bt) {
  return p1b_vec<T, kWavesB>(st, X, pl, P, J, r, B, Z, ws, flag, bt);
}

template <typename T, int NW>
hipError_t p2b_nw(hipStream_t st, const T* X, const PassBPlan& pl, int64_t P, int64_t J, int r, const float* A,
                  double* Y, void* ws, int* flag, const PassLaunch* bl) {
  unsigned gx0, grx0;
  pass2b_grids(pl, &gx0, &grx0);
  const dim3 grid(bl ? bl->gx : gx0, bl ? (unsigned)bl->n : 1u), block(NW * 64);
  const PassDesc* bt = bl ? bl->desc : nullptr;
  float* w = static_cast<float*>(ws);
  const bool vx = pass2b_vx(P);
  if (!(pass_launch_mask() & 1)) {
  } else if (pl.ntn == 1) {
    if (vx)
      hipLaunchKernelGGL((k_pass2b<T, NW, 1, true>), grid, block, 0, st, X, P, J, r, A, w, Y, flag, pl.tiles,
                         pl.chunks, bt);
    else
      hipLaunchKernelGGL((k_pass2b<T, NW, 1, false>), grid, block, 0, st, X, P, J, r, A, w, Y, flag, pl.tiles,
                         pl.chunks, bt);
  } else if constexpr (NW == kWavesB) {  // two rank tiles: four waves only (registers)
    if (vx)
      hipLaunchKernelGGL((k_pass2b<T, NW, 2, true>), grid, block, 0, st, X, P, J, r, A, w, Y, flag, pl.tiles,
                         pl.chunks, bt);
    else
      hipLaunchKernelGGL((k_pass2b<T, NW, 2, false>), grid, block, 0, st, X, P, J, r, A, w, Y, flag, pl.tiles,
                         pl.chunks, bt);
  } else {
    return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (hipEvent_t m = pass_mid_event()) e = hipEventRecord(m, st);
  if (e != hipSuccess) return e;
  if (pl.ntn == 1) return launch_reduce<2, 1, 1>(st, pl, P, J, r, Y, ws, flag, bl);
  return launch_reduce<2, 1, 2>(st, pl, P, J, r, Y, ws, flag, bl);
}

template <typename T>
hipError_t p2s_t(hipStream_t st, const T* X, const PassBPlan& pl, int64_t P, int64_t J, int r, const float* A,
                 double* Y, int* flag, const PassLaunch* bl) {
  const dim3 grid(bl ? bl->gx : (unsigned)pl.tiles, bl ? (unsigned)bl->n : 1u), block(kP2sWaves * 64);
  const PassDesc* bt = bl ? bl->desc : nullptr;
  if (!(pass_launch_mask() & 1)) {
  } else if (pl.ntn == 1) {
    hipLaunchKernelGGL((k_pass2s<T, 1>), grid, block, kP2sLds, st, X, P, J, r, A, Y, flag, bt);
  } else {
    hipLaunchKernelGGL((k_pass2s<T, 2>), grid, block, kP2sLds, st, X, P, J, r, A, Y, flag, bt);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (hipEvent_t m = pass_mid_event()) e = hipEventRecord(m, st);
  return e;
}

template <typename T, int NTN>
hipError_t attr2s() {
  return hipFuncSetAttribute((const void*)k_pass2s<T, NTN>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kP2sLds);
}

template <typename T>
hipError_t p2b_t(hipStream_t st, const T* X, const PassBPlan& pl, int64_t P, int64_t J, int r, const float* A,
                 double* Y, void* ws, int* flag, const PassLaunch* bl) {
  if (pl.staged) return p2s_t<T>(st, X, pl, P, J, r, A, Y, flag, bl);
  if (pl.waves == 8) return p2b_nw<T, 8>(st, X, pl, P, J, r, A, Y, ws, flag, bl);
  return p2b_nw<T, kWavesB>(st, X, pl, P, J, r, A, Y, ws, flag, bl);
}

int chunks_for(int64_t units, int tiles, int cus, int waves, int min_per_wave) {
  int64_t chunks = ((int64_t)cus + tiles - 1) / tiles;
  const int64_t maxc = units / ((int64_t)min_per_wave * waves);
  if (chunks > maxc) chunks = maxc;
  if (chunks < 1) chunks = 1;
  return (int)chunks;
}

}  // namespace

PassBPlan pass1b_finish(PassBPlan pl, int64_t P, int64_t J) {
  (void)J;
  pl.tiles = (int)((P + 32 * pl.vec - 1) / (32 * pl.vec));
  const size_t tilef = (size_t)pl.ntn * pl.vec * 1024;
  pl.ws_bytes = (size_t)pl.tiles * pl.chunks * tilef * sizeof(float);
  return pl;
}

PassBPlan pass2b_finish(PassBPlan pl, int64_t P, int64_t J) {
  (void)P;
  pl.tiles = (int)((J + 31) / 32);
  if (pl.staged) {  // one block per column tile writes its result: no workspace
    pl.chunks = 1;
    pl.waves = kP2sWaves;
    pl.ws_bytes = 256;
    return pl;
  }
  pl.ws_bytes = (size_t)pl.tiles * pl.chunks * pl.ntn * 1024 * sizeof(float);
  return pl;
}

PassBPlan pass1b_plan(int64_t P, int64_t J, int r, int cus) {
  PassBPlan pl;
  pl.ntn = r <= 32 ? 1 : 2;
  // widest row vector that divides P (a tile of 8-row vectors only with one
  // rank tile: its partial tile fills the reduction LDS)
  if (pl.ntn == 1 && P % 8 == 0)
    pl.vec = 8;
  else if (P % 4 == 0)
    pl.vec = 4;
  else
    pl.vec = 1;
  pl.waves = kWavesB;
  pl = pass1b_finish(pl, P, J);
  pl.chunks = chunks_for((J + 15) / 16, pl.tiles, 2 * cus, pl.waves, 2);
  return pass1b_finish(pl, P, J);
}

PassBPlan pass2b_plan(int64_t P, int64_t J, int r, int cus) {
  PassBPlan pl;
  pl.ntn = r <= 32 ? 1 : 2;
  // the staged kernel when its waves need at most two chunks each (measured
  // 8.4 us against 20-24 us on the 1080 x 5760 slice; with few column tiles
  // and long columns the direct kernel's row split wins)
  if (P % 8 == 0 && P <= 2 * kP2sWaves * kP2sRows) {
    pl.staged = 1;
    return pass2b_finish(pl, P, J);
  }
  pl.waves = kWavesB;
  pl = pass2b_finish(pl, P, J);
  pl.chunks = chunks_for((P + 63) / 64, pl.tiles, 2 * cus, pl.waves, 2);
  return pass2b_finish(pl, P, J);
}

void pass1b_grids(const PassBPlan& pl, unsigned* gx, unsigned* grx) {
  *gx = (unsigned)(pl.tiles * ((pl.chunks + 7) / 8) * 8);
  *grx = pl.chunks == 1 ? 0u : (unsigned)(((int64_t)pl.tiles * pl.ntn * pl.vec * 1024 + 255) / 256);
}

void pass2b_grids(const PassBPlan& pl, unsigned* gx, unsigned* grx) {
  if (pl.staged) {
    *gx = (unsigned)pl.tiles;
    *grx = 0u;
    return;
  }
  *gx = (unsigned)(pl.tiles * pl.chunks);
  *grx = pl.chunks == 1 ? 0u : (unsigned)(((int64_t)pl.tiles * pl.ntn * 1024 + 255) / 256);
}

bool pass2b_vx(int64_t P) { return P % 8 == 0; }

hipError_t pass1_bf16(hipStream_t st, const void* X, tt_dtype xdt, const PassBPlan& pl, int64_t P, int64_t J, int r,
                      const float* B, double* Z, void* ws, int* flag, const PassLaunch* bl) {
  if (r < 1 || r > 32 * pl.ntn || pl.ntn > 2 || pl.waves != kWavesB || (bl && (bl->n < 1 || bl->n > 65535)))
    return hipErrorInvalidValue;
  if (pl.chunks < 1 || pl.tiles != (int)((P + 32 * pl.vec - 1) / (32 * pl.vec))) return hipErrorInvalidValue;
  if (pl.vec != 1 && P % pl.vec != 0) return hipErrorInvalidValue;
  if (pl.vec == 8 && pl.ntn != 1) return hipErrorInvalidValue;
  switch (xdt) {
    case TT_F32: return p1b_t(st, static_cast<const float*>(X), pl, P, J, r, B, Z, ws, flag, bl);
    case TT_F64: return p1b_t(st, static_cast<const double*>(X), pl, P, J, r, B, Z, ws, flag, bl);
    case TT_BF16: return p1b_t(st, static_cast<const __hip_bfloat16*>(X), pl, P, J, r, B, Z, ws, flag, bl);
  }
  return hipErrorInvalidValue;
}

hipError_t pass2_bf16(hipStream_t st, const void* X, tt_dtype xdt, const PassBPlan& pl, int64_t P, int64_t J, int r,
                      const float* A, double* Y, void* ws, int* flag, const PassLaunch* bl) {
  if (pl.staged && (P % 8 != 0 || pl.chunks != 1)) return hipErrorInvalidValue;
  if (r < 1 || r > 32 * pl.ntn || pl.ntn > 2 || (bl && (bl->n < 1 || bl->n > 65535)) ||
      (!pl.staged && pl.waves != kWavesB && !(pl.waves == 8 && pl.ntn == 1)))
    return hipErrorInvalidValue;
  if (pl.chunks < 1 || pl.tiles != (int)((J + 31) / 32)) return hipErrorInvalidValue;
  switch (xdt) {
    case TT_F32: return p2b_t(st, static_cast<const float*>(X), pl, P, J, r, A, Y, ws, flag, bl);
    case TT_F64: return p2b_t(st, static_cast<const double*>(X), pl, P, J, r, A, Y, ws, flag, bl);
    case TT_BF16: return p2b_t(st, static_cast<const __hip_bfloat16*>(X), pl, P, J, r, A, Y, ws, flag, bl);
  }
  return hipErrorInvalidValue;
}

hipError_t pass_bf16_setup() {
  hipError_t e = hipSuccess;
#define TT_A2S(T)                                \
  if (e == hipSuccess) e = attr2s<T, 1>();       \
  if (e == hipSuccess) e = attr2s<T, 2>();
  TT_A2S(float)
  TT_A2S(double)
  TT_A2S(__hip_bfloat16)
#undef TT_A2S
  return e;
}

}  // namespace ttk
