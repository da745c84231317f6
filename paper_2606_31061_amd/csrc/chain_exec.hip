// The update's small FP64 chain, run as lists of operations by one workgroup.
//
// Between the two slice passes the update is a sequential chain of small
// dense steps (Algorithm 1): the LQ sweep of the right-orthogonalisation
// (Section 3.4.1), the right interfaces, and for every core the local solve of
// Eq. 5 followed by a thin QR (Section 3.4.2).  Each step is at most a few
// hundred KB, so a step is latency-bound and a kernel launch per step would
// cost more than the step.  Here a host-built list of ChainOp records is
// executed by ONE workgroup of 16 waves (k_chain): consecutive operations are
// separated by a workgroup barrier only.  Contractions large enough to need
// the whole GPU are launched separately by the runtime.
//
// Every operation first copies its operands from global memory into LDS with
// many loads in flight, then computes from LDS:
//   GEMM    C = A B (FP64 v_mfma_f64_16x16x4) with element strides, optional
//           FP32 copy of C.  Operands are staged in k-chunks; each wave keeps
//           at least four independent accumulators so the matrix pipe stays
//           busy.
//   QR      thin QR M = Q R, diag(R) >= 0 (FP64).  Fast path (n <= 32,
//           m <= 512, matrix held in registers): CholeskyQR2 -- Gram matrix,
//           Cholesky factor and its inverse, Q1 = M R1^-1, then the same on
//           Q1, whose Gram matrix I + E is so close to I that its factor is
//           taken to first order in E when |E| <= 1e-7.  When a Cholesky pivot
//           is below (1e-7 ||M||_F)^2 the matrix is ill-conditioned or
//           rank-deficient and the operation falls back to Householder with
//           the identity-reflector rule: a column whose remaining norm is
//           <= tol ||M||_F gets no reflector and R_jj = 0.  `rho` < n caps the
//           number of proper reflectors (later columns get the identity
//           reflector); the runtime uses it where the rank is bounded by
//           construction.
//   NORMG   g normalisation of Section 3.4.1 (G_m absorbs ||g||).
//   COPY    copy of n doubles with an optional FP32 copy.
//   COMMIT  history append and time step, or restore of the old state when
//           the slice was not finite.
#include "tt_internal.h"

namespace ttk {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kCT = kChainThreads;
constexpr int kCW = kCT / 64;

// LDS layout (in doubles; 160 KB).  GEMM and QR operations never overlap in
// time, so their regions alias.  The small QR buffers come first so that
// their addresses fit the LDS instructions' immediate offsets.
constexpr int kLdsTotal = 20480;
// GEMM: staged k-chunks of A and B, split-k partial blocks
constexpr int kStageCap = 14336;
constexpr int kLdsPart = 14336;     // 4352 (4096 padded)
// QR
constexpr int kLdsRow = 0;          // 256: rows of R broadcast to the wave
constexpr int kLdsRed = 256;        // 64: reductions
constexpr int kLdsFlag = 320;       // 8: flags
constexpr int kLdsTau = 328;        // 256: Householder tau
constexpr int kLdsSgn = 584;        // 256: Householder signs
constexpr int kLdsW = 840;          // 1024: Gram matrix, then R2
constexpr int kLdsR1 = 1864;        // 1024: R1
constexpr int kLdsRi = 2888;        // 1056: R1^-1, then R2^-1 (leading dimension 33)
constexpr int kLdsMs = 3944;        // 16448: the matrix (up to 512 rows x 32, odd leading dimension)
constexpr int kQrRows = 512;
constexpr int kMaxHouseholderCols = 256;

// The chain kernels' dynamic LDS.  Operands are addressed by offsets into
// it, so every access compiles to an LDS instruction with a 32-bit address.
extern __shared__ double s_lds[];

constexpr double kCholRel = 1e-7;   // pivot threshold of the fast path, relative to ||M||_F
constexpr double kFirstOrder = 1e-7;

__device__ __forceinline__ int round16(int x) { return (x + 15) & ~15; }

// The thread index, opaque to the optimiser: the chain kernel loops over
// operations, and quantities derived from the thread index would otherwise be
// hoisted out of that loop and kept live (and spilled) across every operation.
__device__ __forceinline__ int tix() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// a / b (returned) and a % b (rem) for 0 <= a < 2^16 and b >= 1, from a
// single-precision reciprocal estimate corrected to the exact quotient (the
// estimate is within one of it; for b >= 2^24 it is below one, as is a / b):
// a few instructions where an integer division takes dozens.
__device__ __forceinline__ int small_div(int a, int b, int& rem) {
  int q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
  int r = a - q * b;
  if (r < 0) {
    --q;
    r += b;
  }
  if (r >= b) {
    ++q;
    r -= b;
  }
  rem = r;
  return q;
}

// use(i, j, ld(i, j)) for every (i, j) of an m x n index space (m, n >= 1)
// in the order of for_each_ij, U elements per thread at a time: the U loads
// are issued together (unconditionally, element (0, 0) standing in past the
// end) before any use, instead of one memory round trip per element.
template <int U, class Ld, class Use>
__device__ __forceinline__ void for_each_ij_ld(int m, int n, Ld ld, Use use) {
  const int tid = tix(), di = kCT % m, dj = kCT / m;
  int i;
  int j = small_div(tid, m, i);
  while (j < n) {
    int ii[U], jj[U];
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ii[u] = i;
      jj[u] = j;
      const bool ok = j < n;
      x[u] = ld(ok ? i : 0, ok ? j : 0);
      i += di;
      j += dj;
      if (i >= m) {
        i -= m;
        ++j;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (jj[u] < n) use(ii[u], jj[u], x[u]);
  }
}

// fn(i, j) for every (i, j) of an m x n index space (m >= 1), the workgroup's
// threads walking i fastest.  The indices advance incrementally, so there is no
// integer division per element.
template <class Fn>
__device__ __forceinline__ void for_each_ij(int m, int n, Fn fn) {
  const int tid = tix(), di = kCT % m, dj = kCT / m;
  int i;
  for (int j = small_div(tid, m, i); j < n;) {
    fn(i, j);
    i += di;
    j += dj;
    if (i >= m) {
      i -= m;
      ++j;
    }
  }
}

__device__ __forceinline__ double read_lane(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Wave reductions without LDS traffic: DPP moves pair lanes within quads
// (xor 1, xor 2) and rows (the half-row and row mirrors), the lane-swap
// instructions pair rows 16 and 32 lanes apart.  Each step adds a lane's value
// and its partner's, in an order that makes every lane of a pair compute the
// same bits (x + y == y + x), so every lane ends with the same total.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// the two values the lanes l and l ^ 16 (l ^ 32) hold, lower row first
template <int D>
__device__ __forceinline__ void row_pair(double v, double& a, double& b) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  if constexpr (D == 16) {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    a = __hiloint2double(h[0], l[0]);
    b = __hiloint2double(h[1], l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a = __hiloint2double(h[0], l[0]);
    b = __hiloint2double(h[1], l[1]);
  }
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  double a, b;
  row_pair<16>(v, a, b);
  v = a + b;
  row_pair<32>(v, a, b);
  return a + b;
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  double a, b;
  row_pair<16>(v, a, b);
  v = fmax(a, b);
  row_pair<32>(v, a, b);
  return fmax(a, b);
}

// Workgroup sum (fixed order: reproducible); every thread gets the total.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kCW; ++i) s += red[i];
  return s;
}

__device__ __forceinline__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < kCW; ++i) s = fmax(s, red[i]);
  return s;
}

// ------------------------------------------------------------------ MFMA on LDS

// A matrix in LDS: element (i, j) at s_lds[off + i * rs + j * cs],
// zero-padded to whole 16-row blocks and 4-value k-steps so that the inner
// loop needs no bounds checks.
struct View {
  int off;
  int rs, cs;
};

// How a wave takes part in a product of nbm x nbn output blocks over nks
// k-steps.  With at least 16 blocks each wave owns blocks w, w+16, ... (at
// most 4), split into P phases over the k-steps when it owns fewer than 3 so
// that at least three chains are in flight.  With fewer blocks and `split`
// the k-steps are divided into ks groups spread over the idle waves and the
// partial blocks are added afterwards in a fixed order; without `split` wave
// w < nb takes block w alone.  Slot q (q < na) accumulates block blk(q) over
// the k-steps s0 + ph(q) + P t below s1.
struct Plan {
  int na, P;   // slots, phases per block (1, 2 or 4)
  int lp;      // log2 P
  int w, nbm, nb;
  int sb;      // the block of a k-split wave, or -1
  int s0, s1;  // k-step range
  int ks, kg;  // k groups, this wave's group (-1: idle)
};

// P is 1, 2 or 4: the slot arithmetic uses shifts (P = 1 << lp)
__device__ __forceinline__ int slot_blk(const Plan& p, int q) { return p.sb >= 0 ? p.sb : p.w + kCW * (q >> p.lp); }
__device__ __forceinline__ int slot_ph(const Plan& p, int q) { return q & (p.P - 1); }

__device__ __forceinline__ Plan wave_plan(int nbm, int nb, int nks, int w, bool split) {
  Plan p;
  p.w = w;
  p.nbm = nbm;
  p.nb = nb;
  p.sb = -1;
  p.na = 0;
  p.P = 1;
  p.lp = 0;
  p.ks = 1;
  p.kg = 0;
  p.s0 = 0;
  p.s1 = nks;
  if (nb >= kCW) {
    const int mine = (nb - w + kCW - 1) / kCW;  // blocks w, w+16, ... below nb (at most 4)
    p.lp = mine >= 3 ? 0 : (mine == 2 ? 1 : 2);
    p.P = 1 << p.lp;
    p.na = mine * p.P;
    return p;
  }
  int ks = split ? kCW / nb : 1;
  if (ks > nks) ks = nks;
  if (ks < 1) ks = 1;
  p.ks = ks;
  if (w < nb * ks) {
    p.kg = small_div(w, nb, p.sb);
    p.s0 = nks * p.kg / ks;
    p.s1 = nks * (p.kg + 1) / ks;
    p.P = 4;
    p.lp = 2;
    p.na = 4;
  } else {
    p.kg = -1;
  }
  return p;
}

// acc[q] += A(block row of slot q, k-steps) B(k-steps, block column of slot q)
// for the slots of plan p over k-steps [s0, s1) (4 values of k per step).
// MFMA operand layout: lane l supplies A(l%16, l/16) and B(l/16, l%16); the
// result holds D(4v + l/16, l%16) in element v.  The slots are independent,
// so the matrix pipe overlaps them.  The operand pointers advance by P
// k-steps; the last, partial round loads only what it uses.
template <int NA>
__device__ __forceinline__ void mma_slots(const View& A, const View& B, const Plan& p, int s0, int s1, v4d* acc) {
  const int lane = tix() & 63;
  const int li = lane & 15, lk = lane >> 4;
  int pa[NA], pb[NA], ph[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    const int b = slot_blk(p, q);
    ph[q] = slot_ph(p, q);
    const int k0 = 4 * (s0 + ph[q]) + lk;
    int bi;
    const int bj = small_div(b, p.nbm, bi);
    pa[q] = A.off + (16 * bi + li) * A.rs + k0 * A.cs;
    pb[q] = B.off + k0 * B.rs + (16 * bj + li) * B.cs;
  }
  const int da = 4 * p.P * A.cs, db = 4 * p.P * B.rs;
  int s = s0;
  for (; s + p.P <= s1; s += p.P) {
    double a[NA], b[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      a[q] = s_lds[pa[q]];
      b[q] = s_lds[pb[q]];
      pa[q] += da;
      pb[q] += db;
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc[q], 0, 0, 0);
  }
  if (s < s1) {
#pragma unroll
    for (int q = 0; q < NA; ++q)
      if (s + ph[q] < s1) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(s_lds[pa[q]], s_lds[pb[q]], acc[q], 0, 0, 0);
  }
}

__device__ __forceinline__ void mma_dispatch(const View& A, const View& B, const Plan& p, int s0, int s1, v4d* acc) {
  switch (p.na) {
    case 1: mma_slots<1>(A, B, p, s0, s1, acc); break;
    case 2: mma_slots<2>(A, B, p, s0, s1, acc); break;
    case 3: mma_slots<3>(A, B, p, s0, s1, acc); break;
    case 4: mma_slots<4>(A, B, p, s0, s1, acc); break;
    default: break;
  }
}

// Finishes a product by storing each block straight from the registers:
// every block's phase slots are added in order.  store(i, j, value) receives
// every output element of the i < M, j < N range.  Ends with a barrier.
// Only for plans without k split (used for small outputs in LDS).
template <class Store>
__device__ __forceinline__ void finish_direct(const Plan& p, int M, int N, const v4d* acc, Store store) {
  const int lane = tix() & 63;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < p.na && slot_ph(p, q) == 0) {
      v4d s = acc[q];
#pragma unroll
      for (int f = 1; f < 4; ++f)
        if (q + f < 4 && f < p.P) s += acc[q + f < 4 ? q + f : 3];
      const int b = slot_blk(p, q);
      int bi;
      const int bj = small_div(b, p.nbm, bi);
      const int i0 = bi * 16, j0 = bj * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 4 * v + (lane >> 4), j = j0 + (lane & 15);
        if (i < M && j < N) store(i, j, s[v]);
      }
    }
  }
  __syncthreads();
}

// Position of element x of finish_lds's buffer: one double of padding after
// every 16, so that a walk along i (stride 16 in the block layout) spreads
// over the LDS banks instead of hitting one.  The padded buffer holds at most
// 64 blocks (17408 doubles).
__device__ __forceinline__ int fpad(int x) { return x + (x >> 4); }

// Finishes a product through LDS: each wave puts its block sums (or, with k
// split, its partial block) in buf[fpad(((kg nb + b) 4 + v) 64 + l)]; after a
// barrier the threads walk the output with i fastest (ifast) or j fastest,
// adding the k groups in order, so that consecutive threads store to
// consecutive addresses.  Ends with a barrier.
template <class Store>
__device__ __forceinline__ void finish_lds(const Plan& p, int M, int N, const v4d* acc, double* buf, bool ifast, Store store) {
  const int lane = tix() & 63;
  if (p.ks == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < p.na && slot_ph(p, q) == 0) {
        v4d s = acc[q];
#pragma unroll
        for (int f = 1; f < 4; ++f)
          if (q + f < 4 && f < p.P) s += acc[q + f < 4 ? q + f : 3];
        const int b = slot_blk(p, q);
#pragma unroll
        for (int v = 0; v < 4; ++v) buf[fpad((b * 4 + v) * 64 + lane)] = s[v];
      }
    }
  } else if (p.kg >= 0) {
    const v4d s = acc[0] + acc[1] + acc[2] + acc[3];
#pragma unroll
    for (int v = 0; v < 4; ++v) buf[fpad(((p.kg * p.nb + p.sb) * 4 + v) * 64 + lane)] = s[v];
  }
  __syncthreads();
  const int rows = 16 * p.nbm, total = p.nb * 256, cols = total / rows;
  // (i, j) of element e, advanced without division
  const int nf = ifast ? rows : cols, df = kCT % nf, ds = kCT / nf;
  int f;
  int sl = small_div(tix(), nf, f);
  for (int e = tix(); e < total; e += kCT) {
    const int i = ifast ? f : sl, j = ifast ? sl : f;
    f += df;
    sl += ds;
    if (f >= nf) {
      f -= nf;
      ++sl;
    }
    if (i < M && j < N) {
      const int b = (i >> 4) + p.nbm * (j >> 4), il = i & 15, jl = j & 15;
      const int o = (b * 4 + (il >> 2)) * 64 + ((il & 3) << 4) + jl;
      double s = 0.0;
      for (int g = 0; g < p.ks; ++g) s += buf[fpad(g * p.nb * 256 + o)];
      store(i, j, s);
    }
  }
  __syncthreads();
}

// C = A B with both operands already in LDS (zero-padded views), nks
// k-steps, at most 64 output blocks; no k split.  Ends with a barrier.
template <class Store>
__device__ __forceinline__ void gemm_lds(int M, int N, int nks, const View& A, const View& B, Store store) {
  const int w = tix() >> 6;
  const int nbm = (M + 15) >> 4, nbn = (N + 15) >> 4;
  const Plan p = wave_plan(nbm, nbm * nbn, nks, w, false);
  v4d acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = (v4d){0.0, 0.0, 0.0, 0.0};
  if (p.na > 0) mma_dispatch(A, B, p, p.s0, p.s1, acc);
  finish_direct(p, M, N, acc, store);
}

// ------------------------------------------------------------------ GEMM (global operands)

struct Gemm {
  int64_t M, N, K;
  const double* A;
  int64_t ars, acs;
  const double* B;
  int64_t brs, bcs;
  double* C;
  int64_t crs, ccs;
  float* C32;
};

// Copies the rows x cols block whose element (i, j) is src[i * rs + j * cs]
// into LDS at dst[i * drs + j * dcs], zero outside i < r_valid, j < c_valid.
// The walk follows the smaller source stride so that the loads coalesce,
// with eight loads in flight per thread.
__device__ __forceinline__ void stage(int dst, int drs, int dcs, int rows, int cols, const double* src, int64_t rs, int64_t cs,
                      int r_valid, int c_valid) {
  constexpr int U = 8;  // loads in flight per thread
  const int total = rows * cols;
  // walk (f, s) = (fast, slow) index; each thread advances by kCT elements
  const bool rfast = rs <= cs;
  const int nf = rfast ? rows : cols;
  const int fv = rfast ? r_valid : c_valid, sv = rfast ? c_valid : r_valid;
  const int64_t fs = rfast ? rs : cs, ss = rfast ? cs : rs;
  const int dfs = rfast ? drs : dcs, dss = rfast ? dcs : drs;
  const int df = kCT % nf, ds = kCT / nf;
  int f;
  int sl = small_div(tix(), nf, f);
  for (int e0 = tix(); e0 < total; e0 += U * kCT) {
    double x[U];
    int fi[U], si[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      fi[u] = f;
      si[u] = sl;
      // unconditional load (element 0 stands in for the padding), so that no
      // load sits in a branch of its own: the compiler then waits for each
      // branch's load before issuing the next one
      const bool ok = e0 + u * kCT < total && f < fv && sl < sv;
      x[u] = src[ok ? f * fs + sl * ss : 0];
      x[u] = ok ? x[u] : 0.0;
      f += df;
      sl += ds;
      if (f >= nf) {
        f -= nf;
        ++sl;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * kCT < total) s_lds[dst + fi[u] * dfs + si[u] * dss] = x[u];
  }
}

// One operand walk of stage_pair: the same order and zero fill as stage, with
// the LDS position of each loaded element kept beside it.
struct StageWalk {
  const double* src;
  int64_t fs, ss;
  int nf, df, ds, fv, sv, dfs, dss, total, dst;
  int f, sl;
  __device__ __forceinline__ StageWalk(int dst_, int drs, int dcs, int rows, int cols, const double* src_, int64_t rs,
                                       int64_t cs, int r_valid, int c_valid) {
    const bool rfast = rs <= cs;
    src = src_;
    nf = rfast ? rows : cols;
    fv = rfast ? r_valid : c_valid;
    sv = rfast ? c_valid : r_valid;
    fs = rfast ? rs : cs;
    ss = rfast ? cs : rs;
    dfs = rfast ? drs : dcs;
    dss = rfast ? dcs : drs;
    df = kCT % nf;
    ds = kCT / nf;
    total = rows * cols;
    dst = dst_;
    sl = small_div(tix(), nf, f);
  }
  template <int U>
  __device__ __forceinline__ void load(int e0, double (&x)[U], int (&o)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = e0 + u * kCT < total;
      o[u] = in ? dst + f * dfs + sl * dss : -1;
      x[u] = (in && f < fv && sl < sv) ? ((const TT_GLOBAL_AS double*)src)[f * fs + sl * ss] : 0.0;
      f += df;
      sl += ds;
      if (f >= nf) {
        f -= nf;
        ++sl;
      }
    }
  }
};

// stage() of both operands of a product: each round issues the loads of A
// and of B before any LDS store, so that small operands cost one memory
// latency instead of two.
__device__ __forceinline__ void stage_pair(StageWalk a, StageWalk b) {
  constexpr int U = 4;  // loads in flight per thread and operand
  const int total = a.total > b.total ? a.total : b.total;
  for (int e0 = tix(); e0 < total; e0 += U * kCT) {
    double xa[U], xb[U];
    int oa[U], ob[U];
    a.load<U>(e0, xa, oa);
    b.load<U>(e0, xb, ob);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (oa[u] >= 0) s_lds[oa[u]] = xa[u];
      if (ob[u] >= 0) s_lds[ob[u]] = xb[u];
    }
  }
}

// Small products (at most kSmallWork multiply-adds per thread): no staging
// and no matrix cores, whose set-up (index walks, LDS round trips, barriers)
// costs several microseconds per operation, more than such a product's
// arithmetic.  Output e = i + M j goes to thread e % (M N) of depth group
// e / (M N): when M N leaves room, the depth is split into G groups (a power of
// two, at most 16), each thread adds its group's terms in k order and the
// groups are added in group order through LDS; otherwise each thread takes
// outputs e, e + kCT, ... over the whole depth.  Consecutive threads walk i,
// the contiguous index of column-major operands.
constexpr int kSmallFma = 65536;
constexpr int kSmallWork = 24;  // multiply-adds per thread
static_assert(kCT == 1024, "small_gemm_fits divides by kCT with a shift");
// log2 of the number of depth groups: at most 16 groups, two outputs' worth
// of threads per group and output, two terms per group
__device__ __forceinline__ int small_gemm_lg(int MN, int K) {
  int lg = 0;
  while (lg < 4 && (MN << (lg + 1)) <= kCT && (2 << lg) <= K) ++lg;
  return lg;
}
__device__ __forceinline__ bool small_gemm_fits(int MN, int K) {
  const int lg = small_gemm_lg(MN, K);
  return ((MN + kCT - 1) >> 10) * ((K + (1 << lg) - 1) >> lg) <= kSmallWork;
}
__device__ __forceinline__ void small_gemm(const Gemm& g, int M, int N, int K) {
  const int tid = tix();
  const int MN = M * N;
  const int lg = small_gemm_lg(MN, K), G = 1 << lg;
  auto dot = [&](int e, int k0, int k1) {
    int i;
    const int j = small_div(e, M, i);
    const double* a = g.A + i * (int)g.ars;
    const double* b = g.B + j * (int)g.bcs;
    const int as = (int)g.acs, bs = (int)g.brs;
    double acc = 0.0;
#pragma unroll 4
    for (int k = k0; k < k1; ++k) acc = fma(a[k * as], b[k * bs], acc);
    return acc;
  };
  auto store = [&](int e, double v) {
    int i;
    const int j = small_div(e, M, i);
    const int o = i * (int)g.crs + j * (int)g.ccs;
    if (g.C) g.C[o] = v;
    if (g.C32) g.C32[o] = (float)v;
  };
  if (G == 1) {
    for (int e = tid; e < MN; e += kCT) store(e, dot(e, 0, K));
  } else {
    double* part = s_lds + kLdsPart;  // G * MN <= kCT doubles
    const int kper = (K + G - 1) >> lg;
    int e;
    const int grp = small_div(tid, MN, e);
    if (grp < G) {
      const int k0 = grp * kper, k1 = k0 + kper < K ? k0 + kper : K;
      part[tid] = dot(e, k0, k1);
    }
    __syncthreads();
    if (tid < MN) {
      double v = 0.0;
      for (int q = 0; q < G; ++q) v += part[q * MN + tid];
      store(tid, v);
    }
  }
  __syncthreads();
}

// Products with n <= 32 and depth <= 32 that small_gemm does not take: B goes
// to LDS (zero beyond n, up to whole 8-column groups), and thread t computes
// row i = t % M of one group of 8 output columns, adding the depth in k order
// (A read once per row and k; B read from LDS, the same address across the
// wave).  Consecutive threads take consecutive rows, so column-major A and C
// are read and written along their contiguous index.
constexpr int kRowCols = 8;
__device__ __forceinline__ void rowblock_gemm(const Gemm& g, int M, int N, int K) {
  const int tid = tix();
  double* Bs = s_lds + kLdsPart;  // K x 32, column-major, leading dimension 32
  const int ng = (N + kRowCols - 1) / kRowCols;
  const int ncols = ng * kRowCols;
  for (int e = tid; e < 32 * ncols; e += kCT) {
    const int k = e & 31, j = e >> 5;
    const bool ok = k < K && j < N;
    const double v = g.B[ok ? k * g.brs + j * g.bcs : 0];
    Bs[e] = ok ? v : 0.0;
  }
  __syncthreads();
  const int ars = g.ars, acs = g.acs;
  for (int t = tid; t < M * ng; t += kCT) {
    int i;
    const int grp = small_div(t, M, i);
    const int j0 = grp * kRowCols;
    const double* a = g.A + i * ars;
    const double* b = Bs + 32 * j0;
    double acc[kRowCols];
#pragma unroll
    for (int c = 0; c < kRowCols; ++c) acc[c] = 0.0;
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
      const double x = a[k * acs];
#pragma unroll
      for (int c = 0; c < kRowCols; ++c) acc[c] = fma(x, b[k + 32 * c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < kRowCols; ++c) {
      if (j0 + c < N) {
        const int o = i * g.crs + (j0 + c) * g.ccs;
        if (g.C) g.C[o] = acc[c];
        if (g.C32) g.C32[o] = (float)acc[c];
      }
    }
  }
  __syncthreads();
}

// C = A B from global operands.  The output is cut into tiles of at most
// 64 blocks; for each tile the needed rows of A and columns of B go through
// LDS one k-chunk at a time.
__device__ __forceinline__ void wg_gemm(const Gemm& g) {
  const int M = (int)g.M, N = (int)g.N, K = (int)g.K;
  if (M <= 0 || N <= 0) {
    __syncthreads();
    return;
  }
  if ((int64_t)M * N * K <= kSmallFma && small_gemm_fits(M * N, K)) {
    small_gemm(g, M, N, K);
    return;
  }
  if (N <= 32 && K <= 32) {
    rowblock_gemm(g, M, N, K);
    return;
  }
  if (M <= 32 && K <= 32) {  // the same on C^T = B^T A^T
    rowblock_gemm(Gemm{g.N, g.M, g.K, g.B, g.bcs, g.brs, g.A, g.acs, g.ars, g.C, g.ccs, g.crs, g.C32}, N, M, K);
    return;
  }
  const int w = tix() >> 6;
  const int nbm_all = (M + 15) >> 4, nbn_all = (N + 15) >> 4;
  const int nks = (K + 3) >> 2;
  const int TR = nbm_all < 64 ? nbm_all : 64;
  const int TC = nbn_all < 64 / TR ? nbn_all : 64 / TR;
  double* part = s_lds + kLdsPart;
  for (int cb0 = 0; cb0 < nbn_all; cb0 += TC) {
    for (int rb0 = 0; rb0 < nbm_all; rb0 += TR) {
      const int nbm = nbm_all - rb0 < TR ? nbm_all - rb0 : TR;
      const int nbn = nbn_all - cb0 < TC ? nbn_all - cb0 : TC;
      const int Mp = 16 * nbm, Np = 16 * nbn;
      const int Mv = M - 16 * rb0, Nv = N - 16 * cb0;
      const Plan p = wave_plan(nbm, nbm * nbn, nks, w, true);
      // without k split the whole LDS may hold operands (the blocks are
      // collected at offset 0 afterwards); with it the partial blocks need
      // their own region
      int chunk = (p.ks == 1 ? kLdsTotal : kStageCap) / (4 * (Mp + Np));  // k-steps staged at a time
      if (chunk < 1) chunk = 1;
      v4d acc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = (v4d){0.0, 0.0, 0.0, 0.0};
      const double* Ag = g.A + (int64_t)16 * rb0 * g.ars;
      const double* Bg = g.B + (int64_t)16 * cb0 * g.bcs;
      for (int c0 = 0; c0 < nks; c0 += chunk) {
        const int c1 = c0 + chunk < nks ? c0 + chunk : nks;
        const int kc = 4 * (c1 - c0);
        const int As = 0;            // Mp x kc, element (i, k) at i + Mp k
        const int Bs = Mp * kc;      // kc x Np, element (k, j) at j + Np k
        __syncthreads();
        stage_pair(StageWalk(As, 1, Mp, Mp, kc, Ag + (int64_t)4 * c0 * g.acs, g.ars, g.acs, Mv, K - 4 * c0),
                   StageWalk(Bs, Np, 1, kc, Np, Bg + (int64_t)4 * c0 * g.brs, g.brs, g.bcs, K - 4 * c0, Nv));
        __syncthreads();
        const int s0 = p.s0 > c0 ? p.s0 : c0, s1 = p.s1 < c1 ? p.s1 : c1;
        if (p.na > 0 && s0 < s1) {
          const View A{As, 1, Mp}, B{Bs, Np, 1};
          mma_dispatch(A, B, p, s0 - c0, s1 - c0, acc);
        }
      }
      __syncthreads();
      const int64_t ro = (int64_t)16 * rb0, co = (int64_t)16 * cb0;
      finish_lds(p, Mv, Nv, acc, p.ks == 1 ? s_lds : part, g.crs <= g.ccs, [&](int i, int j, double v) {
        const int64_t o = (ro + i) * g.crs + (co + j) * g.ccs;
        if (g.C) g.C[o] = v;
        if (g.C32) g.C32[o] = (float)v;
      });
    }
  }
}

// ------------------------------------------------------------------ Cholesky

// 1/sqrt(d) for d > 0: hardware estimate and NEWTON Newton steps (two give
// full FP64).
template <int NEWTON>
__device__ __forceinline__ double rsqrt_pos(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
#pragma unroll
  for (int i = 0; i < NEWTON; ++i) y = y * fma(-h * y, y, 1.5);
  return y;
}

// Cholesky factor of the 32 x 32 symmetric matrix W (LDS, column-major) and
// its inverse, by four waves (one per SIMD); every thread of the workgroup
// calls it, passes the same barriers and receives the same status.  Wave w
// (w < 4) owns rows 8w .. 8w+7: lane c < 32 holds their entries in column c
// of W, turned into column c of R (W = R^T R, R upper triangular); lane
// 32 + c holds them in column c of X, which starts as the identity and
// receives the same elimination steps, so that it ends as R^-T.  Step j
// scales row j by 1/sqrt(pivot) and removes R(j,:)^T R(j,:) from the rows
// below.  The steps go in blocks of four rows inside one wave: the few
// entries a step needs come from single lanes (v_readlane), and that wave
// also updates its own rows below the block.  It then publishes the block's
// rows through LDS, by lane and transposed (the multipliers of row i,
// R(jb..jb+3, i), in one place), and after a barrier the waves that own rows
// further down apply the block's four updates to them.  The published rows
// alternate between two buffers (the Householder scratch, idle here), so
// one barrier per block suffices.  Every entry receives the same fused
// multiply-adds in the same order as in a one-wave elimination.  Only
// pivots of the first n columns are tested against thr2.  Writes R (zeros
// below the diagonal, leading dimension 32) and R^-1 (leading dimension 33);
// R may alias W.  NB = 8 factors the leading 8 columns only (beyond n <= 8,
// W is the identity, whose columns no step changes): that stays in wave 0
// and needs no barrier before the last.  NEWTON = 1 leaves the pivots'
// square roots good to about 1e-10 relative, which suffices when a second
// CholeskyQR pass corrects the factor: R and R^-1 are exact inverses of each
// other either way.
template <int NB, int NEWTON>
__device__ __forceinline__ bool chol_inv(const double* W, double* R, double* Ri, double thr2, int n) {
  constexpr int RW = 8;  // rows per wave
  const int tid = tix(), lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  int c = lane & 31;
  // opaque to the optimiser: keeps the identity set-up below from being
  // hoisted out of the operation loop
  asm volatile("" : "+v"(c));
  const bool xh = lane >= 32;
  int* okw = reinterpret_cast<int*>(s_lds + kLdsFlag) + 4;  // one status per wave
  double v[RW];
  bool ok = true;
  if (w < 4) {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int i = RW * w + r;
      double x = W[i + 32 * c];
      asm volatile("" : "+v"(x));  // loaded by every lane: no branch around the load
      v[r] = xh ? (i == c ? 1.0 : 0.0) : x;
    }
  }
#pragma unroll
  for (int jb = 0; jb < NB; jb += 4) {
    const int q = jb / RW, o = jb % RW;     // owning wave, its first row of the block
    const bool others = NB > RW * (q + 1);  // rows below in later waves
    const bool odd = (jb / 4) & 1;
    double* bl = s_lds + (odd ? kLdsTau : kLdsRow);        // bl[64 k + lane] = row jb + k
    double* bt = s_lds + kLdsSgn + (odd ? 128 : 0);        // bt[4 i + k] = R(jb + k, i)
    if (w == q) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double d = read_lane(v[o + j], jb + j);
        ok = ok && (jb + j >= n || d > thr2);
        v[o + j] *= rsqrt_pos<NEWTON>(d);
#pragma unroll
        for (int i = j + 1; i < 4; ++i) v[o + i] = fma(-read_lane(v[o + j], jb + i), v[o + j], v[o + i]);
      }
      if (others) {
#pragma unroll
        for (int k = 0; k < 4; ++k) bl[64 * k + lane] = v[o + k];
        if (!xh) {
          double2* t = reinterpret_cast<double2*>(bt + 4 * lane);
          t[0] = make_double2(v[o], v[o + 1]);
          t[1] = make_double2(v[o + 2], v[o + 3]);
        }
      }
      // this wave's own rows below the block
#pragma unroll
      for (int i = o + 4; i < RW; ++i) {
        if (RW * q + i < NB) {
          const double r0 = read_lane(v[o], RW * q + i), r1 = read_lane(v[o + 1], RW * q + i);
          const double r2 = read_lane(v[o + 2], RW * q + i), r3 = read_lane(v[o + 3], RW * q + i);
          v[i] = fma(-r0, v[o], v[i]);
          v[i] = fma(-r1, v[o + 1], v[i]);
          v[i] = fma(-r2, v[o + 2], v[i]);
          v[i] = fma(-r3, v[o + 3], v[i]);
        }
      }
    }
    if (others) {
      __syncthreads();
      if (w > q && w < NB / RW) {
        const double l0 = bl[lane], l1 = bl[64 + lane], l2 = bl[128 + lane], l3 = bl[192 + lane];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const double2* t = reinterpret_cast<const double2*>(bt + 4 * (RW * w + r));
          const double2 a01 = t[0], a23 = t[1];
          v[r] = fma(-a01.x, l0, v[r]);
          v[r] = fma(-a01.y, l1, v[r]);
          v[r] = fma(-a23.x, l2, v[r]);
          v[r] = fma(-a23.y, l3, v[r]);
        }
      }
    }
  }
  if (w < 4) {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int i = RW * w + r;
      double* dst = xh ? Ri + c + 33 * i : R + i + 32 * c;
      *dst = (xh || i <= c) ? v[r] : 0.0;
    }
    if (lane == 0) okw[w] = ok ? 1 : 0;
  }
  __syncthreads();
  return (okw[0] & okw[1] & okw[2] & okw[3]) != 0;
}

// The factorisation stops after the leading NB columns when n <= NB: beyond
// n, W is the identity, whose columns no elimination step changes.
template <int NEWTON>
__device__ __forceinline__ bool chol_inv32(const double* W, double* R, double* Ri, double thr2, int n) {
  if (n <= 8) return chol_inv<8, NEWTON>(W, R, Ri, thr2, n);
  return chol_inv<32, NEWTON>(W, R, Ri, thr2, n);
}

// R = R2 R1 for the upper triangular 32 x 32 factors of CholeskyQR2 in LDS
// (R2 in W, then R1; column-major, leading dimension 32, zeros below the
// diagonal, the identity beyond n), written to the n x n matrix R (leading
// dimension n).  The blocks (0,0), (0,1) and (1,1) go to the matrix cores,
// one wave each, over the k range in which neither triangle vanishes; wave
// 3 writes the zero block (1,0).  Every thread calls it; the caller's
// barrier publishes R.
__device__ __forceinline__ void upper_product(const double* W, const double* R1, int n, double* R) {
  const int tid = tix(), lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (wv >= 4) return;
  const int bi = wv >= 2 ? 1 : 0, bj = (wv == 1 || wv == 2) ? 1 : 0;
  const int k0 = wv == 2 ? 4 : 0, k1 = wv == 0 ? 4 : (wv == 3 ? 0 : 8);
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int kc = k0; kc < k1; ++kc) {
    const double a = W[(16 * bi + li) + 32 * (4 * kc + lk)];
    const double b = R1[(4 * kc + lk) + 32 * (16 * bj + li)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 16 * bi + 4 * v + lk, col = 16 * bj + li;
    if (row < n && col < n) R[row + n * col] = acc[v];
  }
}

// ------------------------------------------------------------------ QR

struct Qr {
  int m, n, rho;
  const double* M;
  int64_t mrs, mcs;
  double* Q;
  int64_t qrs, qcs;
  double* R;     // n x n column-major, or null
  double* aux;   // m * n doubles of device scratch
  double tol;
};

// Applies the reflector H_j = I - t v v^T (v_j = 1, v_i = A(i, j) below) to
// columns j+1 .. n-1 of A, row-parallel, for tall matrices in device memory:
// every thread owns rows.  Per block of at most 32 columns, one pass forms
// the dot products v^T A(:, c), four columns at a time (one coalesced load
// per column and row), each added lane-wise in the wave (fixed shuffle
// order) and then in wave order through LDS (part: 17 x 33 doubles); a
// second pass updates the block.  Few registers, so it sits next to the rest
// of the chain without spilling.
__device__ __forceinline__ void hh_apply_rows(double* A, int m, int n, int lda, int j, double t, double* part) {
  const int tid = tix(), lane = tid & 63, wid = tid >> 6;
  const double* cj = A + (int64_t)j * lda;
  const int nc = n - j - 1;
  if (nc <= 0) {  // still a barrier: the caller's thread-0 writes must land
    __syncthreads();
    return;
  }
  for (int cb = 0; cb < nc; cb += 32) {  // blocks of at most 32 columns
    const int nb = nc - cb < 32 ? nc - cb : 32;
    double* a0 = A + (int64_t)(j + 1 + cb) * lda;  // column j+1+cb
    for (int q = 0; q < nb; q += 4) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int i = j + 1 + tid; i < m; i += kCT) {
        const double vi = cj[i];
        const double* row = a0 + i + (int64_t)q * lda;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q + u < nb) acc[u] = fma(vi, row[(int64_t)u * lda], acc[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double d = wave_sum(acc[u]);
        if (lane == 0 && q + u < nb) part[wid * 33 + q + u] = d;
      }
    }
    __syncthreads();
    if (tid < nb) {
      double* a = a0 + j + (int64_t)tid * lda;
      double d = *a;
      for (int w = 0; w < kCW; ++w) d += part[w * 33 + tid];
      const double tw = t * d;
      part[kCW * 33 + tid] = tw;
      *a -= tw;
    }
    __syncthreads();
    const double* tw = part + kCW * 33;
    for (int i = j + 1 + tid; i < m; i += kCT) {
      const double vi = cj[i];
      double* row = a0 + i;
      int c = 0;
      for (; c + 4 <= nb; c += 4) {
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = row[(int64_t)(c + u) * lda];
#pragma unroll
        for (int u = 0; u < 4; ++u) row[(int64_t)(c + u) * lda] = fma(-tw[c + u], vi, x[u]);
      }
      for (; c < nb; ++c) row[(int64_t)c * lda] = fma(-tw[c], vi, row[(int64_t)c * lda]);
    }
    __syncthreads();
  }
}

// Householder factorisation of the m x n column-major matrix A (leading
// dimension lda) in place: R on and above the diagonal, the reflector vectors
// (unit leading entry implied) below it, tau[j] their scalars,
// H_j = I - tau_j v_j v_j^T, H_j x = beta e_1 with beta = -sign(x_1) ||x||.
// Column j gets the identity reflector (tau = 0, zeroed from the diagonal
// down) when its remaining norm is <= thr, or once rho proper reflectors
// have been built (the rank is then exhausted: without pivoting the
// independent columns may be anywhere, so this counts reflectors, not
// columns).
__device__ __forceinline__ void hh_factor(double* A, int m, int n, int lda, double thr, int rho, bool need_r, double* tau,
                          double* red, bool rows_par) {
  const int tid = tix(), lane = tid & 63, wid = tid >> 6;
  int built = 0;
  for (int j = 0; j < n; ++j) {
    double* cj = A + (int64_t)j * lda;
    double nrm = 0.0;
    if (built >= rho) {
      // rank exhausted: every remaining column gets the identity reflector,
      // which only zeroes that column from the diagonal down (R) and touches
      // no other column, so all of them are done at once
      if (need_r)
        for (int c = j; c < n; ++c) {
          double* cc = A + (int64_t)c * lda;
          for (int i = c + tid; i < m; i += kCT) cc[i] = 0.0;
        }
      for (int c = j + tid; c < n; c += kCT) tau[c] = 0.0;
      __syncthreads();
      return;
    }
    if (built < rho) {
      double p = 0.0;
      for (int i = j + tid; i < m; i += kCT) {
        const double x = cj[i];
        p = fma(x, x, p);
      }
      nrm = sqrt(block_sum(p, red));
    }
    const double alpha = cj[j];
    __syncthreads();
    if (!(nrm > thr)) {
      for (int i = j + tid; i < m; i += kCT) cj[i] = 0.0;
      if (tid == 0) tau[j] = 0.0;
      __syncthreads();
      continue;
    }
    ++built;
    const double beta = alpha >= 0.0 ? -nrm : nrm;
    const double scal = 1.0 / (alpha - beta);
    for (int i = j + 1 + tid; i < m; i += kCT) cj[i] *= scal;
    const double t = (beta - alpha) / beta;
    __syncthreads();
    if (tid == 0) {
      cj[j] = beta;
      tau[j] = t;
    }
    if (built == rho && !need_r) {
      // the last proper reflector: the columns after j only receive identity
      // reflectors and are overwritten when Q is formed, so updating them
      // serves R alone
      for (int c = j + 1 + tid; c < n; c += kCT) tau[c] = 0.0;
      __syncthreads();
      return;
    }
    if (rows_par) {
      hh_apply_rows(A, m, n, lda, j, t, s_lds + kLdsMs);
      continue;
    }
    for (int c = j + 1 + wid; c < n; c += kCW) {
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

// Overwrites the factored A with the thin Q = H_0 ... H_{n-1} [I; 0]
// (backward accumulation; the caller applies the column signs).  Columns with
// the identity reflector (tau = 0) hold no reflector data, so they all become
// unit vectors without a barrier between them; both kinds of column are found
// from bit masks of tau (one ballot per 64 columns, the same in every wave),
// and each proper reflector costs two barriers.
__device__ __forceinline__ void hh_form_q(double* A, int m, int n, int lda, const double* tau, bool rows_par) {
  const int tid = tix(), lane = tid & 63, wid = tid >> 6;
  for (int jw = 0; jw <= (n - 1) >> 6; ++jw)
    for (uint64_t mk = __ballot(64 * jw + lane < n && tau[64 * jw + lane] == 0.0); mk != 0; mk &= mk - 1) {
      const int j = 64 * jw + __ffsll((long long)mk) - 1;
      double* cj = A + (int64_t)j * lda;
      for (int i = tid; i < m; i += kCT) cj[i] = (i == j) ? 1.0 : 0.0;
    }
  __syncthreads();
  for (int jw = (n - 1) >> 6; jw >= 0; --jw)
  for (uint64_t mk = __ballot(64 * jw + lane < n && tau[64 * jw + lane] != 0.0); mk != 0;) {
    const int b = 63 - __clzll((long long)mk);
    mk &= ~(1ull << b);
    const int j = 64 * jw + b;
    const double t = tau[j];
    double* cj = A + (int64_t)j * lda;
    if (rows_par) {
      hh_apply_rows(A, m, n, lda, j, t, s_lds + kLdsMs);
    } else {
      for (int c = j + 1 + wid; c < n; c += kCW) {
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
    for (int i = tid; i < m; i += kCT) {
      double v;
      if (i < j) v = 0.0;
      else if (i == j) v = 1.0 - t;
      else v = -t * cj[i];
      cj[i] = v;
    }
    __syncthreads();  // the next reflector reads this column
  }
}

__device__ __forceinline__ void hh_form_q_wy(const Qr& q, const double* A, const double* tau, const double* sgn);

// Householder QR of q.M, already copied into A (column-major, leading
// dimension lda; LDS or the scratch buffer).
__device__ __forceinline__ void householder_qr(const Qr& q, double* A, int lda) {
  double* tau = s_lds + kLdsTau;
  double* sgn = s_lds + kLdsSgn;
  double* red = s_lds + kLdsRed;
  const int m = q.m, n = q.n, tid = tix();
  const bool rows_par = A == q.aux;  // tall: the matrix is in device memory (lda = m)
  double p = 0.0;
  if (rows_par) {
    const int64_t total = (int64_t)m * n;
#pragma unroll 8
    for (int64_t e = tid; e < total; e += kCT) p = fma(A[e], A[e], p);
  } else {
    for_each_ij(m, n, [&](int i, int j) {
      const double x = A[i + (int64_t)j * lda];
      p = fma(x, x, p);
    });
  }
  const double fro = sqrt(block_sum(p, red));
  hh_factor(A, m, n, lda, q.tol * fro, q.rho, q.R != nullptr, tau, red, rows_par);
  for (int j = tid; j < n; j += kCT) sgn[j] = (tau[j] != 0.0 && A[j + (int64_t)j * lda] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  if (q.R) {
    for_each_ij(n, n, [&](int i, int j) { q.R[i + n * j] = (i <= j) ? sgn[i] * A[i + (int64_t)j * lda] : 0.0; });
  }
  __syncthreads();
  if (rows_par && n <= 32) {  // tall: Q in compact WY form, written to q.Q
    hh_form_q_wy(q, A, tau, sgn);
    return;
  }
  hh_form_q(A, m, n, lda, tau, rows_par);
  for_each_ij(m, n, [&](int i, int j) {
    const double v = A[i + (int64_t)j * lda];
    q.Q[i * q.qrs + j * q.qcs] = sgn[j] < 0.0 ? -v : v;
  });
  __syncthreads();
}

// The 32 x 32 stripe M(r0 .. r0 + 31, 0 .. 31) of an m x n matrix (zero
// outside it) into this wave's LDS tile, element (r, c) at tile[32 r + (c ^ r)]
// (the XOR keeps both the row and the column walks on distinct banks).  The
// lanes walk M's contiguous index (rows when mrs <= mcs, columns otherwise),
// so each load instruction reads whole cache lines; all 16 loads of a lane are
// issued before the first is used.  One CU reads only some tens of GB/s, so
// loads that touch 16 lines for 32 bytes each cost several microseconds per
// tall matrix.
__device__ __forceinline__ void load_tile(const double* M, int mrs, int mcs, int r0, int m, int n, double* tile) {
  const int lane = tix() & 63, a = lane & 31, h = lane >> 5;
  const bool rows = mrs <= mcs;  // lanes walk rows (a = row) or columns (a = column)
  double x[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = rows ? a : 2 * k + h, c = rows ? 2 * k + h : a;
    const bool ok = r0 + r < m && c < n;
    x[k] = M[ok ? (unsigned)((r0 + r) * mrs + c * mcs) : 0u];
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = rows ? a : 2 * k + h, c = rows ? 2 * k + h : a;
    const bool ok = r0 + r < m && c < n;
    tile[32 * r + (c ^ r)] = ok ? x[k] : 0.0;
  }
  __builtin_amdgcn_wave_barrier();
}

// Row fragments f[s][cb] = X(4 s + l / 16, 16 cb + l % 16) and column fragments
// g[t][kc] = X(16 t + l % 16, 4 kc + l / 16) of a wave's tile (see load_tile).
__device__ __forceinline__ void tile_rows(const double* tile, double (&f)[8][2]) {
  const int lane = tix() & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int r = 4 * s + lk, c = 16 * cb + li;
      f[s][cb] = tile[32 * r + (c ^ r)];
    }
  __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ void tile_cols(const double* tile, double (&g)[2][8]) {
  const int lane = tix() & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
      const int r = 16 * t + li, c = 4 * kc + lk;
      g[t][kc] = tile[32 * r + (c ^ r)];
    }
  __builtin_amdgcn_wave_barrier();
}

// Partial Gram blocks of a wave's 32-row stripe held in row fragments
// f[s][cb] = X(r0 + 4s + l/16, 16 cb + l%16): blocks (0,0), (1,0), (1,1) of
// X^T X go to part[(3 w + blk) * 256 + 64 v + l] (zero for a stripe wholly
// below the matrix, live = false); after a barrier the first nlive stripes
// (those that hold rows; the rest are zero) are added in order into W
// (32 x 32, column-major, mirrored).
__device__ __forceinline__ void stripe_gram(const double (&f)[8][2], bool live, int nlive, double* part, double* W) {
  const int tid = tix(), lane = tid & 63, w = tid >> 6;
  v4d g00 = {0.0, 0.0, 0.0, 0.0}, g10 = g00, g11 = g00;
  if (live) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      g00 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[s][0], f[s][0], g00, 0, 0, 0);
      g10 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[s][1], f[s][0], g10, 0, 0, 0);
      g11 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[s][1], f[s][1], g11, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    part[(3 * w + 0) * 256 + 64 * v + lane] = g00[v];
    part[(3 * w + 1) * 256 + 64 * v + lane] = g10[v];
    part[(3 * w + 2) * 256 + 64 * v + lane] = g11[v];
  }
  __syncthreads();
  if (tid < 768) {
    const int blk = tid >> 8, e = tid & 255, v = e >> 6, l = e & 63;
    const int bi = blk == 0 ? 0 : 1, bj = blk == 2 ? 1 : 0;
    double sum = 0.0;
#pragma unroll 4
    for (int ww = 0; ww < nlive; ++ww) sum += part[(3 * ww + blk) * 256 + e];
    const int i = 16 * bi + 4 * v + (l >> 4), j = 16 * bj + (l & 15);
    W[i + 32 * j] = sum;
    if (bi != bj) W[j + 32 * i] = sum;
  }
  __syncthreads();
}

// CholeskyQR2 of an m x n matrix (m <= 512, n <= 32) with the data in
// registers: wave w owns rows 32w .. 32w+31.  Row fragments (rows along the
// MFMA k index) feed the Gram matrices, column fragments (rows along the
// block index) feed Q = M R^-1.  Only the 32 x 32 Gram matrices and
// triangular factors go through LDS, plus one transposition of Q1.  Returns
// false, with nothing written, when a pivot test fails.
__device__ __forceinline__ bool cholqr2_reg(const Qr& q) {
  const int tid = tix(), lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int m = q.m, n = q.n;
  const int r0 = 32 * w;
  const bool live = r0 < m;  // this wave's stripe holds rows of the matrix
  double* part = s_lds + kLdsMs;  // 12288 doubles, then the Q1 transposition (ld = 513)
  double* W = s_lds + kLdsW;
  double* R1 = s_lds + kLdsR1;
  double* Ri = s_lds + kLdsRi;
  double* red = s_lds + kLdsRed;
  constexpr int ldq = 513;
  // 32-bit offsets (chain_fits32): one address register per load and no
  // 64-bit multiplications
  const int mrs = (int)q.mrs, mcs = (int)q.mcs;

  // pass 1: W = M^T M from row fragments, read through the wave's LDS tile
  double* tile = part + 1024 * w;
  double f[8][2];
  double g[2][8];  // the column fragments for Q1 = M R1^-1, kept from the same read
  if (live) {
    load_tile(q.M, mrs, mcs, r0, m, n, tile);
    tile_rows(tile, f);
    tile_cols(tile, g);
  } else {
#pragma unroll
    for (int s = 0; s < 8; ++s) f[s][0] = f[s][1] = 0.0;
  }
  __syncthreads();
  stripe_gram(f, live, (m + 31) >> 5, part, W);
  {
    const int i = tid & 31, j = tid >> 5;
    if (i >= n || j >= n) W[i + 32 * j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  {  // the trace of W (= ||M||_F^2) and the factor
    double fro2 = 0.0;
#pragma unroll 4
    for (int i = 0; i < n; ++i) fro2 += W[i * 33];
    if (!chol_inv32<1>(W, R1, Ri, kCholRel * kCholRel * fro2, n)) return false;
  }

  // Q1 = M R1^-1: column fragments of M (from the first read), result in
  // row-fragment order: block (t, cb) element v is Q1(r0 + 16t + 4v + l/16, 16cb + l%16)
  {
    v4d acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[t][cb] = (v4d){0.0, 0.0, 0.0, 0.0};
    if (live) {
      // R^-1 is upper triangular: column block 0 only meets k < 16
#pragma unroll
      for (int kc = 0; kc < 8; ++kc) {
        const double b1 = Ri[(4 * kc + lk) + 33 * (16 + li)];
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[t][kc], b1, acc[t][1], 0, 0, 0);
        if (kc < 4) {
          const double b0 = Ri[(4 * kc + lk) + 33 * li];
#pragma unroll
          for (int t = 0; t < 2; ++t) acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[t][kc], b0, acc[t][0], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) f[4 * t + v][cb] = acc[t][cb][v];
  }
  __syncthreads();  // Ri is read above and rewritten below
  // pass 2: W = Q1^T Q1 = I + E
  stripe_gram(f, live, (m + 31) >> 5, part, W);
  const int i = tid & 31, j = tid >> 5;
  const double e = (i < n && j < n) ? W[i + 32 * j] - (i == j ? 1.0 : 0.0) : 0.0;
  const double emax = block_max(fabs(e), red);
  if (emax <= kFirstOrder) {
    // R2 = I + U and R2^-1 = I - U to first order, U the upper triangle of E
    // with half its diagonal (error O(|E|^2)); R2 overwrites W
    const double u = (i < j) ? e : (i == j ? 0.5 * e : 0.0);
    W[i + 32 * j] = (i == j ? 1.0 : 0.0) + u;
    Ri[i + 33 * j] = (i == j ? 1.0 : 0.0) - u;
    __syncthreads();
  } else {
    if (i >= n || j >= n) W[i + 32 * j] = (i == j) ? 1.0 : 0.0;
    __syncthreads();
    if (!chol_inv32<2>(W, W, Ri, 0.25, n)) return false;
  }
  // Q = Q1 R2^-1: Q1 goes through LDS to become column fragments
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) part[(r0 + 4 * s + lk) + ldq * (16 * cb + li)] = f[s][cb];
  __syncthreads();
  {
    v4d acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[t][cb] = (v4d){0.0, 0.0, 0.0, 0.0};
    if (live) {
#pragma unroll
      for (int kc = 0; kc < 8; ++kc) {
        const double b1 = Ri[(4 * kc + lk) + 33 * (16 + li)];
        const double b0 = kc < 4 ? Ri[(4 * kc + lk) + 33 * li] : 0.0;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const double a = part[(r0 + 16 * t + li) + ldq * (4 * kc + lk)];
          if (kc < 4) acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc[t][0], 0, 0, 0);
          acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc[t][1], 0, 0, 0);
        }
      }
    }
    // Q goes back through LDS so that the global stores are contiguous
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) part[(r0 + 16 * t + 4 * v + lk) + ldq * (16 * cb + li)] = acc[t][cb][v];
    __syncthreads();
    // the threads walk Q along its contiguous index (f) and step the indices
    // incrementally: no integer division per element
    const bool ifast = q.qrs <= q.qcs;
    const int nf = ifast ? m : n, ns = ifast ? n : m, df = kCT % nf, ds = kCT / nf;
    int f;
    for (int sl = small_div(tid, nf, f); sl < ns;) {
      const int row = ifast ? f : sl, col = ifast ? sl : f;
      q.Q[row * q.qrs + col * q.qcs] = part[row + ldq * col];
      f += df;
      sl += ds;
      if (f >= nf) {
        f -= nf;
        ++sl;
      }
    }
  }
  if (q.R) upper_product(W, R1, n, q.R);
  __syncthreads();
  return true;
}

// Gram contributions of one 32-row stripe held as row fragments (see
// stripe_gram), added to the wave's accumulators.
__device__ __forceinline__ void gram_acc(const double (&f)[8][2], v4d& g00, v4d& g10, v4d& g11) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    g00 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[s][0], f[s][0], g00, 0, 0, 0);
    g10 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[s][1], f[s][0], g10, 0, 0, 0);
    g11 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[s][1], f[s][1], g11, 0, 0, 0);
  }
}

// The waves' Gram accumulators added in wave order into W (32 x 32, mirrored).
__device__ __forceinline__ void gram_reduce(const v4d& g00, const v4d& g10, const v4d& g11, double* part,
                                            double* W) {
  const int tid = tix(), lane = tid & 63, w = tid >> 6;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    part[(3 * w + 0) * 256 + 64 * v + lane] = g00[v];
    part[(3 * w + 1) * 256 + 64 * v + lane] = g10[v];
    part[(3 * w + 2) * 256 + 64 * v + lane] = g11[v];
  }
  __syncthreads();
  if (tid < 768) {
    const int blk = tid >> 8, e = tid & 255, v = e >> 6, l = e & 63;
    const int bi = blk == 0 ? 0 : 1, bj = blk == 2 ? 1 : 0;
    double sum = 0.0;
#pragma unroll
    for (int ww = 0; ww < kCW; ++ww) sum += part[(3 * ww + blk) * 256 + e];
    const int i = 16 * bi + 4 * v + (l >> 4), j = 16 * bj + (l & 15);
    W[i + 32 * j] = sum;
    if (bi != bj) W[j + 32 * i] = sum;
  }
  __syncthreads();
}

// Product of a 32-row stripe (column fragments g: g[t][kc] is the element
// (16 t + l % 16, 4 kc + l / 16)) with the upper-triangular Ri (LDS, leading
// dimension 33); result in row-fragment order (see cholqr2_reg).
__device__ __forceinline__ void stripe_times_upper(const double (&g)[2][8], const double* Ri, double (&f)[8][2]) {
  const int lane = tix() & 63, li = lane & 15, lk = lane >> 4;
  v4d acc[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) acc[t][cb] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kc = 0; kc < 8; ++kc) {
    const double b1 = Ri[(4 * kc + lk) + 33 * (16 + li)];
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[t][kc], b1, acc[t][1], 0, 0, 0);
    if (kc < 4) {
      const double b0 = Ri[(4 * kc + lk) + 33 * li];
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[t][kc], b0, acc[t][0], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) f[4 * t + v][cb] = acc[t][cb][v];
}

// Q of a factored tall matrix (A = the scratch copy, m x n column-major,
// n <= 32) in compact WY form: with the proper reflectors v_1..v_nb (columns
// j_1 < .. < j_nb of A below the diagonal, unit at row j_k, zero above),
// H_1 .. H_nb = I - V T V^T with T upper triangular (T_kk = tau_k,
// T(1:k-1, k) = -tau_k T(1:k-1, 1:k-1) (V^T V)(1:k-1, k)), so
// Q(i, c) = delta_ic - sum_k V(i, k) W(k, c),  W = T V(0:n-1, :)^T.
// V^T V comes from 32-row stripes by MFMA (as in the Gram passes below), T
// from one wave, and Q from the stripes again by MFMA, written to q.Q with
// the column signs.  Two passes over A instead of two per reflector.
__device__ __forceinline__ void hh_form_q_wy(const Qr& q, const double* A, const double* tau, const double* sgn) {
  const int tid = tix(), lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int m = q.m, n = q.n;
  int* jl = reinterpret_cast<int*>(s_lds + kLdsRow);  // proper columns, in order
  double* G = s_lds + kLdsW;    // V^T V (32 x 32)
  double* T = s_lds + kLdsR1;   // T (32 x 32, column-major)
  double* Wm = s_lds + kLdsRi;  // W (32 x 32, leading dimension 33; rows past nb zero)
  double* part = s_lds + kLdsMs;
  const uint64_t mk = __ballot(lane < n && tau[lane] != 0.0);
  const int nb = __popcll(mk);
  if (tid < n && ((mk >> tid) & 1)) jl[__popcll(mk & ((1ull << tid) - 1))] = tid;
  __syncthreads();
  int jc[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) jc[cb] = 16 * cb + li < nb ? jl[16 * cb + li] : -1;
  {
    v4d g00 = {0.0, 0.0, 0.0, 0.0}, g10 = g00, g11 = g00;
#pragma unroll 1
    for (int r0 = 32 * w; r0 < m; r0 += kQrRows) {
      double f[8][2];
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          const int row = r0 + 4 * s + lk, j = jc[cb];
          double a = row == j ? 1.0 : 0.0;
          if (j >= 0 && row > j && row < m) a = A[row + (int64_t)m * j];  // only lanes that need it load
          f[s][cb] = a;
        }
      gram_acc(f, g00, g10, g11);
    }
    __syncthreads();
    gram_reduce(g00, g10, g11, part, G);
  }
  // V(0:n-1, :) into LDS, then T by one wave
  {
    const int c = tid & 31, k = tid >> 5;
    if (c < n && k < nb) {
      const int j = jl[k];
      part[c + 32 * k] = c < j ? 0.0 : (c == j ? 1.0 : A[c + (int64_t)m * j]);
    }
  }
  if (tid < 64) {
    for (int k = 0; k < nb; ++k) {
      const double tk = tau[jl[k]];
      double acc = 0.0;
      for (int qq = lane; qq < k; ++qq) acc += T[lane + 32 * qq] * G[qq + 32 * k];
      if (lane < 32) T[lane + 32 * k] = lane < k ? -tk * acc : (lane == k ? tk : 0.0);
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  {
    const int k = tid & 31, c = tid >> 5;
    double acc = 0.0;
    if (k < nb && c < n)
      for (int qq = k; qq < nb; ++qq) acc += T[k + 32 * qq] * part[c + 32 * qq];
    Wm[k + 33 * c] = acc;
  }
  __syncthreads();
#pragma unroll 1
  for (int r0 = 32 * w; r0 < m; r0 += kQrRows) {
    double g[2][8];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kc = 0; kc < 8; ++kc) {
        const int row = r0 + 16 * t + li, kq = 4 * kc + lk;
        const int j = kq < nb ? jl[kq] : -1;
        double a = row == j ? 1.0 : 0.0;
        if (j >= 0 && row > j && row < m) a = A[row + (int64_t)m * j];
        g[t][kc] = a;
      }
    v4d acc[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[t][cb] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 8; ++kc) {
      const double b0 = Wm[(4 * kc + lk) + 33 * li], b1 = Wm[(4 * kc + lk) + 33 * (16 + li)];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[t][kc], b0, acc[t][0], 0, 0, 0);
        acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[t][kc], b1, acc[t][1], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          const int row = r0 + 16 * t + 4 * v + lk, col = 16 * cb + li;
          if (row < m && col < n) {
            const double x = (row == col ? 1.0 : 0.0) - acc[t][cb][v];
            q.Q[row * q.qrs + col * q.qcs] = sgn[col] < 0.0 ? -x : x;
          }
        }
  }
  __syncthreads();
}

// Stores a wave's 32-row stripe held as row fragments (f[s][cb] is the
// element (4 s + l / 16, 16 cb + l % 16) of rows r0 .. r0 + 31) to
// X[row * rs + col * cs] (row < m, col < n) through the wave's own 32 x 32 LDS
// tile, whose columns are XOR-swizzled by the row so that the fragment writes
// and the column reads both spread over the banks: the global stores then run
// along rows, contiguous for a column-major X.
__device__ __forceinline__ void store_stripe(const double (&f)[8][2], double* tile, int r0, int m, int n, double* X,
                                             int64_t rs, int64_t cs) {
  const int lane = tix() & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int r = 4 * s + lk, c = 16 * cb + li;
      tile[r * 32 + (c ^ r)] = f[s][cb];
    }
  __builtin_amdgcn_wave_barrier();
  const int r = lane & 31, row = r0 + r, h = lane >> 5;
  if (row < m) {
    double* xr = X + row * rs + h * cs;
    const int64_t step = 2 * cs;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int c = 2 * k + h;
      if (c < n) xr[k * step] = tile[r * 32 + (c ^ r)];
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// CholeskyQR2 of a tall m x n matrix (m > 512, n <= 32), streamed in
// 512-row stripes (wave w takes rows 32 w .. 32 w + 31 of each stripe):
//   A: W = M^T M,                   R1 = chol(W), Ri = R1^-1
//   B: Q1 = M Ri into aux,          W = Q1^T Q1, R2 = chol(W) (first order
//                                   when W is within kFirstOrder of I)
//   C: Q = Q1 R2^-1,                R = R2 R1.
// Q1 goes to the op's scratch, so M (which Q may alias) is intact until
// pass C; returns false, with Q and R untouched, when a pivot test fails.
__device__ __forceinline__ bool cholqr2_tall(const Qr& q) {
  const int tid = tix(), lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int m = q.m, n = q.n;
  const int nst = (m + kQrRows - 1) / kQrRows;
  double* part = s_lds + kLdsMs;
  double* W = s_lds + kLdsW;
  double* R1 = s_lds + kLdsR1;
  double* Ri = s_lds + kLdsRi;
  double* red = s_lds + kLdsRed;
  double* Q1 = q.aux;  // m x n column-major

  // A stripe's loads (unconditional, see stage(): entries outside the
  // matrix read the nearest one inside) and, apart from them, the zeroing of
  // those entries, so that the next stripe's loads go out before this one's
  // arithmetic waits on its own
  auto fetch_rows = [&](const double* A, int ars, int acs, int st, double (&f)[8][2]) {
    const int r0 = kQrRows * st + 32 * w;
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int row = min(r0 + 4 * s + lk, m - 1), col = min(16 * cb + li, n - 1);
        f[s][cb] = A[(unsigned)(row * ars + col * acs)];
      }
  };
  auto mask_rows = [&](int st, double (&f)[8][2]) {
    const int r0 = kQrRows * st + 32 * w;
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int row = r0 + 4 * s + lk, col = 16 * cb + li;
        f[s][cb] = (row < m && col < n) ? f[s][cb] : 0.0;
      }
  };
  auto fetch_cols = [&](const double* A, int ars, int acs, int st, double (&g)[2][8]) {
    const int r0 = kQrRows * st + 32 * w;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kc = 0; kc < 8; ++kc) {
        const int row = min(r0 + 16 * t + li, m - 1), col = min(4 * kc + lk, n - 1);
        g[t][kc] = A[(unsigned)(row * ars + col * acs)];
      }
  };
  auto mask_cols = [&](int st, double (&g)[2][8]) {
    const int r0 = kQrRows * st + 32 * w;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int kc = 0; kc < 8; ++kc) {
        const int row = r0 + 16 * t + li, col = 4 * kc + lk;
        g[t][kc] = (row < m && col < n) ? g[t][kc] : 0.0;
      }
  };
  // A stripe read along M's contiguous index (lanes as in load_tile, the
  // addresses of entries outside the matrix clamped), then, once its loads
  // have landed, written to the wave's LDS tile with those entries zeroed:
  // for the one of passes A and B whose fragments, read straight from M,
  // would take 32 bytes of each of 16 cache lines per load
  auto fetch_tile = [&](const double* A, int ars, int acs, int st, double (&x)[16]) {
    const int a = lane & 31, h = lane >> 5, r0 = kQrRows * st + 32 * w;
    const bool rows = ars <= acs;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int r = rows ? a : 2 * k + h, c = rows ? 2 * k + h : a;
      const int row = min(r0 + r, m - 1), col = min(c, n - 1);
      x[k] = A[(unsigned)(row * ars + col * acs)];
    }
  };
  auto put_tile = [&](int st, int ars, int acs, const double (&x)[16], double* tile) {
    const int a = lane & 31, h = lane >> 5, r0 = kQrRows * st + 32 * w;
    const bool rows = ars <= acs;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int r = rows ? a : 2 * k + h, c = rows ? 2 * k + h : a;
      tile[32 * r + (c ^ r)] = (r0 + r < m && c < n) ? x[k] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
  };
  auto pad_identity = [&]() {
    const int i = tid & 31, j = tid >> 5;
    if (i >= n || j >= n) W[i + 32 * j] = (i == j) ? 1.0 : 0.0;
  };

  // pass A
  {
    v4d g00 = {0.0, 0.0, 0.0, 0.0}, g10 = g00, g11 = g00;
    const int mrs = (int)q.mrs, mcs = (int)q.mcs;
    if (mrs <= mcs) {  // row fragments straight from a column-major M would be scattered
      double x[16], f[8][2];
      double* tile = part + 1024 * w;
      fetch_tile(q.M, mrs, mcs, 0, x);
#pragma unroll 1
      for (int st = 0; st < nst; ++st) {
        put_tile(st, mrs, mcs, x, tile);
        if (st + 1 < nst) fetch_tile(q.M, mrs, mcs, st + 1, x);  // in flight during the Gram
        tile_rows(tile, f);
        gram_acc(f, g00, g10, g11);
      }
    } else {
      double fa[8][2], fb[8][2];
      fetch_rows(q.M, mrs, mcs, 0, fa);
#pragma unroll 1
      for (int st = 0; st < nst; st += 2) {  // two stripes in turn, the next one's loads in flight
        if (st + 1 < nst) fetch_rows(q.M, mrs, mcs, st + 1, fb);
        mask_rows(st, fa);
        gram_acc(fa, g00, g10, g11);
        if (st + 2 < nst) fetch_rows(q.M, mrs, mcs, st + 2, fa);
        if (st + 1 < nst) {
          mask_rows(st + 1, fb);
          gram_acc(fb, g00, g10, g11);
        }
      }
    }
    __syncthreads();
    gram_reduce(g00, g10, g11, part, W);
  }
  pad_identity();
  __syncthreads();
  {  // the trace of W (= ||M||_F^2) and the factor
    double fro2 = 0.0;
#pragma unroll 4
    for (int i = 0; i < n; ++i) fro2 += W[i * 33];
    if (!chol_inv32<1>(W, R1, Ri, kCholRel * kCholRel * fro2, n)) return false;
  }

  // pass B
  {
    v4d h00 = {0.0, 0.0, 0.0, 0.0}, h10 = h00, h11 = h00;
    double ga[2][8], f[8][2];
    auto finish = [&](const double (&g)[2][8], int st) {
      stripe_times_upper(g, Ri, f);
      gram_acc(f, h00, h10, h11);
      store_stripe(f, part + 1024 * w, kQrRows * st + 32 * w, m, n, Q1, 1, m);
    };
    const int mrs = (int)q.mrs, mcs = (int)q.mcs;
    if (mrs > mcs) {  // column fragments straight from a row-major M would be scattered
      double* tile = part + 1024 * w;
#pragma unroll 1
      for (int st = 0; st < nst; ++st) {
        double x[16];
        fetch_tile(q.M, mrs, mcs, st, x);
        put_tile(st, mrs, mcs, x, tile);
        tile_cols(tile, ga);
        finish(ga, st);  // its stores stage through the same tile, after the reads above
      }
    } else {
#pragma unroll 1
      for (int st = 0; st < nst; ++st) {
        fetch_cols(q.M, mrs, mcs, st, ga);
        mask_cols(st, ga);
        finish(ga, st);
      }
    }
    __syncthreads();  // Ri is read above and rewritten below; Q1 complete
    gram_reduce(h00, h10, h11, part, W);
  }
  {
    const int i = tid & 31, j = tid >> 5;
    const double e = (i < n && j < n) ? W[i + 32 * j] - (i == j ? 1.0 : 0.0) : 0.0;
    const double emax = block_max(fabs(e), red);
    if (emax <= kFirstOrder) {
      const double u = (i < j) ? e : (i == j ? 0.5 * e : 0.0);
      W[i + 32 * j] = (i == j ? 1.0 : 0.0) + u;
      Ri[i + 33 * j] = (i == j ? 1.0 : 0.0) - u;
      __syncthreads();
    } else {
      pad_identity();
      __syncthreads();
      if (!chol_inv32<2>(W, W, Ri, 0.25, n)) return false;
    }
  }

  // pass C
  {
    double ga[2][8], f[8][2];
    auto finish = [&](const double (&g)[2][8], int st) {
      stripe_times_upper(g, Ri, f);
      const int r0 = kQrRows * st + 32 * w;
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          const int row = r0 + 4 * s + lk, col = 16 * cb + li;
          if (row < m && col < n) q.Q[row * q.qrs + col * q.qcs] = f[s][cb];
        }
    };
    double gb[2][8];
    fetch_cols(Q1, 1, m, 0, ga);
#pragma unroll 1
    for (int st = 0; st < nst; st += 2) {
      if (st + 1 < nst) fetch_cols(Q1, 1, m, st + 1, gb);
      mask_cols(st, ga);
      finish(ga, st);
      if (st + 2 < nst) fetch_cols(Q1, 1, m, st + 2, ga);
      if (st + 1 < nst) {
        mask_cols(st + 1, gb);
        finish(gb, st + 1);
      }
    }
  }
  if (q.R) upper_product(W, R1, n, q.R);
  __syncthreads();
  return true;
}

// Thin QR of a matrix whose proper reflectors are capped at one (rho = 1,
// e.g. the last core's local solution, which is always rank one), R not
// wanted: the Householder factorisation with the identity-reflector rule
// builds exactly one proper reflector H = I - t v v^T, at the first column j0
// whose norm from the diagonal down exceeds tol ||M||_F (identity reflectors
// before it change no other column), so Q = H [I; 0] in closed form:
// Q(:, j) = e_j for j < j0 and e_j - t v v_j for j >= j0, column j0 negated
// when R(j0, j0) = beta < 0.  One pass over M for the column norms, v staged
// in LDS (M may alias Q), one pass writing Q.  m <= kRank1Rows.
constexpr int kRank1Rows = 16384;
__device__ __forceinline__ void rank1_qr(const Qr& q) {
  const int tid = tix(), lane = tid & 63, wid = tid >> 6;
  const int m = q.m, n = q.n;
  double* cf = s_lds + kLdsTau;  // full column norms^2
  double* cr = s_lds + kLdsSgn;  // norms^2 from the diagonal down
  double* v = s_lds + kLdsMs;    // the reflector (m values)
  double* sc = s_lds + kLdsRed;  // [0] t, [1] sign of column j0, [2] j0 (as double)
  for (int j = wid; j < n; j += kCW) {
    const double* col = q.M + (int64_t)j * q.mcs;
    double pf = 0.0, pr = 0.0;
    int i = lane;
    // eight rows per lane in flight, added in row order as in the remainder
    for (; i + 7 * 64 < m; i += 8 * 64) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = col[(int64_t)(i + 64 * u) * q.mrs];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        pf = fma(x[u], x[u], pf);
        if (i + 64 * u >= j) pr = fma(x[u], x[u], pr);
      }
    }
    for (; i < m; i += 64) {
      const double x = col[(int64_t)i * q.mrs];
      pf = fma(x, x, pf);
      if (i >= j) pr = fma(x, x, pr);
    }
    pf = wave_sum(pf);
    pr = wave_sum(pr);
    if (lane == 0) {
      cf[j] = pf;
      cr[j] = pr;
    }
  }
  __syncthreads();
  if (tid == 0) {
    double fro2 = 0.0;
    for (int j = 0; j < n; ++j) fro2 += cf[j];
    const double thr = q.tol * sqrt(fro2);
    int j0 = n;
    for (int j = 0; j < n && j0 == n; ++j)
      if (sqrt(cr[j]) > thr) j0 = j;
    double t = 0.0, flip = 1.0, scal = 0.0;
    if (j0 < n) {
      const double alpha = q.M[j0 * q.mrs + (int64_t)j0 * q.mcs];
      const double nrm = sqrt(cr[j0]);
      const double beta = alpha >= 0.0 ? -nrm : nrm;
      scal = 1.0 / (alpha - beta);
      t = (beta - alpha) / beta;
      flip = beta < 0.0 ? -1.0 : 1.0;
    }
    sc[0] = t;
    sc[1] = flip;
    sc[2] = (double)j0;
    sc[3] = scal;
  }
  __syncthreads();
  const double t = sc[0], flip = sc[1], scal = sc[3];
  const int j0 = (int)sc[2];
  if (j0 < n) {
#pragma unroll 4
    for (int i = tid; i < m; i += kCT)
      v[i] = (i < j0) ? 0.0 : (i == j0 ? 1.0 : q.M[i * q.mrs + (int64_t)j0 * q.mcs] * scal);
  }
  __syncthreads();
  for_each_ij(m, n, [&](int i, int j) {
    double val = (i == j) ? 1.0 : 0.0;
    if (j >= j0 && j0 < n) {
      val -= t * v[i] * v[j];
      if (j == j0) val *= flip;
    }
    q.Q[i * q.qrs + j * q.qcs] = val;
  });
  __syncthreads();
}

// Thin QR with the proper reflectors capped at 2 <= rho <= 4 (a local
// solution of rank at most rho), R not wanted: Householder builds its rho
// proper reflectors from the first rho columns alone (when none of them
// takes an identity reflector), and the other columns only receive identity
// reflectors, so Q = H_1 .. H_rho [I; 0] = E - V T V_top^T (compact WY form:
// V the m x rho reflectors, unit diagonal, T upper triangular, V_top the
// first n rows of V), column j negated where R(j, j) = beta_j < 0.  The
// m x rho panel goes to LDS (the whole matrix is read once, for ||M||_F), one
// wave factors it and forms T with wave reductions only (lane l owns rows
// l, l + 64, ...: no lane reads what another wrote), and Q is written in one
// pass, wave w taking columns w, w + 16, ... and each lane its rows.  Returns
// false, with nothing written, when one of the first rho columns would take
// an identity reflector (the general path then decides).  m rho <= kMsDoubles.
constexpr int kMsDoubles = 16448;
constexpr int kSmallRho = 4;
constexpr int kPanelRows = 8;  // rows per lane of the register panel (m <= 512)
__device__ __forceinline__ bool small_capped_qr(const Qr& q) {
  const int tid = tix(), lane = tid & 63, w = tid >> 6;
  const int m = q.m, n = q.n, rho = q.rho;
  double* Pn = s_lds + kLdsMs;        // the panel, column-major, leading dimension m
  double* red = s_lds + kLdsRow;      // block sums
  double* U = s_lds + kLdsW;          // U = T V_top^T, kSmallRho x n (leading dimension kSmallRho)
  double* sc = s_lds + kLdsTau;       // beta[4], T (4 x 4, column-major) at 8, status at 24
  // panel into LDS and ||M||_F^2
  double p = 0.0;
  for_each_ij_ld<8>(
      m, n, [&](int i, int j) { return q.M[i * q.mrs + j * q.mcs]; },
      [&](int i, int j, double x) {
        p = fma(x, x, p);
        if (j < rho) Pn[i + m * j] = x;
      });
  const double thr = q.tol * sqrt(block_sum(p, red));
  if (w == 0) {
    double tau[kSmallRho] = {0.0, 0.0, 0.0, 0.0};
    bool ok = true;
    if (m <= 64 * kPanelRows) {
      // the panel in registers: lane l holds rows l + 64 k, k < kPanelRows
      double P[kPanelRows][kSmallRho];
#pragma unroll
      for (int k = 0; k < kPanelRows; ++k)
#pragma unroll
        for (int j = 0; j < kSmallRho; ++j) {
          const int i = lane + 64 * k;
          P[k][j] = (i < m && j < rho) ? Pn[i + m * j] : 0.0;
        }
#pragma unroll
      for (int j = 0; j < kSmallRho; ++j) {
        if (j >= rho || !ok) break;
        double s2 = 0.0;
#pragma unroll
        for (int k = 0; k < kPanelRows; ++k)
          if (lane + 64 * k >= j) s2 = fma(P[k][j], P[k][j], s2);
        const double nrm = sqrt(wave_sum(s2));
        ok = nrm > thr;  // uniform: every lane has the same sum
        if (!ok) break;
        const double alpha = read_lane(P[0][j], j);  // row j < 64 lives in lane j
        const double beta = alpha >= 0.0 ? -nrm : nrm;
        const double scal = 1.0 / (alpha - beta);
        tau[j] = (beta - alpha) / beta;
#pragma unroll
        for (int k = 0; k < kPanelRows; ++k) {
          const int i = lane + 64 * k;
          if (i == j) P[k][j] = 1.0;
          else if (i > j) P[k][j] *= scal;
        }
        if (lane == 0) sc[j] = beta;
#pragma unroll
        for (int c2 = j + 1; c2 < kSmallRho; ++c2) {
          if (c2 >= rho) break;
          double d = 0.0;
#pragma unroll
          for (int k = 0; k < kPanelRows; ++k)
            if (lane + 64 * k >= j) d = fma(P[k][j], P[k][c2], d);
          const double f = tau[j] * wave_sum(d);
#pragma unroll
          for (int k = 0; k < kPanelRows; ++k)
            if (lane + 64 * k >= j) P[k][c2] = fma(-f, P[k][j], P[k][c2]);
        }
      }
      // the reflectors back to LDS for the other waves
#pragma unroll
      for (int k = 0; k < kPanelRows; ++k)
#pragma unroll
        for (int j = 0; j < kSmallRho; ++j) {
          const int i = lane + 64 * k;
          if (i < m && j < rho) Pn[i + m * j] = P[k][j];
        }
      __builtin_amdgcn_wave_barrier();
    } else {
      for (int j = 0; j < rho && ok; ++j) {
        double* cj = Pn + m * j;
        double s2 = 0.0;
        for (int i = lane; i < m; i += 64)
          if (i >= j) s2 = fma(cj[i], cj[i], s2);
        const double nrm = sqrt(wave_sum(s2));
        ok = nrm > thr;  // uniform: every lane has the same sum
        if (!ok) break;
        const double alpha = cj[j];
        __builtin_amdgcn_wave_barrier();  // every lane has read cj[j] before its owner rewrites it
        const double beta = alpha >= 0.0 ? -nrm : nrm;
        const double scal = 1.0 / (alpha - beta);
        tau[j] = (beta - alpha) / beta;
        for (int i = lane; i < m; i += 64)
          if (i >= j) cj[i] = (i == j) ? 1.0 : cj[i] * scal;
        if (lane == 0) sc[j] = beta;
        // H_j on the panel's later columns: c -= tau_j v (v^T c)
        for (int c2 = j + 1; c2 < rho; ++c2) {
          double* cc = Pn + m * c2;
          double d = 0.0;
          for (int i = lane; i < m; i += 64)
            if (i >= j) d = fma(cj[i], cc[i], d);
          const double f = tau[j] * wave_sum(d);
          for (int i = lane; i < m; i += 64)
            if (i >= j) cc[i] = fma(-f, cj[i], cc[i]);
        }
      }
    }
    if (ok) {
      // T: T_bb = tau_b, T(0:b, b) = -tau_b T(0:b, 0:b) V(:, 0:b)^T v_b, from the
      // pair products V(:, a)^T V(:, b), a < b (V(i, a) = 0 above row a)
      double g[kSmallRho][kSmallRho];
#pragma unroll
      for (int b = 1; b < kSmallRho; ++b)
#pragma unroll
        for (int a2 = 0; a2 < b; ++a2) {
          double d = 0.0;
          if (b < rho)
            for (int i = lane; i < m; i += 64)
              if (i >= b) d = fma(Pn[i + m * a2], Pn[i + m * b], d);
          g[a2][b] = wave_sum(d);
        }
      double T[kSmallRho][kSmallRho];
#pragma unroll
      for (int b = 0; b < kSmallRho; ++b)
#pragma unroll
        for (int a2 = 0; a2 < kSmallRho; ++a2) T[a2][b] = 0.0;
#pragma unroll
      for (int b = 0; b < kSmallRho; ++b) {
        if (b >= rho) break;
        T[b][b] = tau[b];
#pragma unroll
        for (int a2 = 0; a2 < b; ++a2) {
          double acc = 0.0;
#pragma unroll
          for (int c = a2; c < b; ++c) acc += T[a2][c] * g[c][b];
          T[a2][b] = -tau[b] * acc;
        }
      }
      if (lane < kSmallRho * kSmallRho) {
        const int a2 = lane & 3, b = lane >> 2;
        double v = 0.0;
#pragma unroll
        for (int e = 0; e < kSmallRho * kSmallRho; ++e)
          if (e == lane) v = T[e & 3][e >> 2];
        sc[8 + a2 + kSmallRho * b] = v;
      }
    }
    if (lane == 0) sc[24] = ok ? 1.0 : 0.0;
  }
  __syncthreads();
  if (sc[24] == 0.0) return false;  // uniform
  const double* T = sc + 8;
  // U = T V_top^T (kSmallRho x n, rows >= rho zero); V_top(c, b) = 0 for c < b, 1 for c == b
  for (int e = tid; e < kSmallRho * n; e += kCT) {
    const int a2 = e & 3, c = e >> 2;
    double acc = 0.0;
    for (int b = a2; b < rho; ++b) {
      const double vcb = c < b ? 0.0 : (c == b ? 1.0 : Pn[c + m * b]);
      acc = fma(T[a2 + kSmallRho * b], vcb, acc);
    }
    U[e] = acc;
  }
  __syncthreads();
  for (int i = lane; i < m; i += 64) {
    double pv[kSmallRho];
#pragma unroll
    for (int a2 = 0; a2 < kSmallRho; ++a2)
      pv[a2] = a2 >= rho ? 0.0 : (i < a2 ? 0.0 : (i == a2 ? 1.0 : Pn[i + m * a2]));
    for (int c = w; c < n; c += kCW) {
      double val = (i == c) ? 1.0 : 0.0;
#pragma unroll
      for (int a2 = 0; a2 < kSmallRho; ++a2) val = fma(-pv[a2], U[a2 + kSmallRho * c], val);
      if (c < rho && sc[c] < 0.0) val = -val;
      q.Q[i * q.qrs + c * q.qcs] = val;
    }
  }
  __syncthreads();
  return true;
}

// The completion of a tall QR capped at rho < n (see wg_qr): C = E - Q_rho W^T
// into Q's columns rho..n-1, W = Q_rho(rho..n-1, :).  Laid out like
// rowblock_gemm: -W^T goes to LDS (zero beyond rho and nc), thread t takes
// row i = t % m of one group of 8 completion columns and walks the depth in
// k order from the identity entry (the same FMA sequence for every layout),
// several rows of Q_rho in flight.  The columns read (k < rho) and written
// (rho and beyond) are disjoint.
__device__ __forceinline__ void capped_completion(const Qr& q) {
  const int tid = tix();
  const int m = q.m, n = q.n, rho = q.rho;
  const int nc = n - rho;
  double* Bs = s_lds + kLdsPart;  // Bs[k + 32 jc] = -W(jc, k)
  for (int e = tid; e < 32 * 32; e += kCT) {
    const int k = e & 31, jc = e >> 5;
    const bool ok = k < rho && jc < nc;
    const double v = q.Q[ok ? (rho + jc) * q.qrs + k * q.qcs : 0];
    Bs[e] = ok ? -v : 0.0;
  }
  __syncthreads();
  double* C = q.Q + (int64_t)rho * q.qcs;
  const int ng = (nc + kRowCols - 1) / kRowCols;
  for (int t = tid; t < m * ng; t += kCT) {
    int i;
    const int j0 = small_div(t, m, i) * kRowCols;
    const double* a = q.Q + i * q.qrs;
    const double* b = Bs + 32 * j0;
    double acc[kRowCols];
#pragma unroll
    for (int c = 0; c < kRowCols; ++c) acc[c] = (i == rho + j0 + c) ? 1.0 : 0.0;
#pragma unroll 8
    for (int k = 0; k < rho; ++k) {
      const double x = a[k * q.qcs];
#pragma unroll
      for (int c = 0; c < kRowCols; ++c) acc[c] = fma(x, b[k + 32 * c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < kRowCols; ++c)
      if (j0 + c < nc) C[i * q.qrs + (j0 + c) * q.qcs] = acc[c];
  }
  __syncthreads();
}

// The completion of a tall QR capped at rho < n in one pass, when it is well
// conditioned: with W = Q_rho(rho..n-1, :) (nc x rho) the completion
// C = E - Q_rho W^T has the Gram matrix C^T C = I - W W^T exactly (Q_rho
// orthonormal), so its Cholesky factor R (nc x nc, one wave, every pivot
// above 1/4, i.e. no column of C shorter than 1/2) orthonormalises it without
// reading C: Q_c = C R^-1 = E R^-1 - Q_rho (W^T R^-1).  Row i of E R^-1 is row
// i - rho of R^-1 for rho <= i < n and zero elsewhere, so the row-blocked loop
// of capped_completion starts from it and adds Q_rho times B = -W^T R^-1.
// Returns false, with nothing written, when a pivot is 1/4 or less.
__device__ __forceinline__ bool capped_completion_closed(const Qr& q) {
  const int tid = tix();
  const int m = q.m, n = q.n, rho = q.rho;
  const int nc = n - rho;
  double* Wm = s_lds + kLdsMs;    // Wm[jc + 32 k] = W(jc, k)
  double* G = s_lds + kLdsW;      // I - W W^T, identity beyond nc
  double* R = s_lds + kLdsR1;
  double* Ri = s_lds + kLdsRi;    // R^-1, leading dimension 33
  double* Bs = s_lds + kLdsPart;  // Bs[k + 32 jc] = B(k, jc)
  {
    const int jc = tid & 31, k = tid >> 5;
    const bool ok = jc < nc && k < rho;
    const double v = q.Q[ok ? (rho + jc) * q.qrs + k * q.qcs : 0];
    Wm[jc + 32 * k] = ok ? v : 0.0;
  }
  __syncthreads();
  {
    const int i = tid & 31, j = tid >> 5;
    double v = (i == j) ? 1.0 : 0.0;
    if (i < nc && j < nc)
      for (int k = 0; k < rho; ++k) v = fma(-Wm[i + 32 * k], Wm[j + 32 * k], v);
    G[i + 32 * j] = v;
  }
  __syncthreads();
  if (!chol_inv32<2>(G, R, Ri, 0.25, nc)) return false;
  {
    const int k = tid & 31, jc = tid >> 5;
    double v = 0.0;
    if (k < rho && jc < nc)
      for (int l = 0; l <= jc; ++l) v = fma(-Wm[l + 32 * k], Ri[l + 33 * jc], v);
    Bs[k + 32 * jc] = v;
  }
  __syncthreads();
  double* C = q.Q + (int64_t)rho * q.qcs;
  const int ng = (nc + kRowCols - 1) / kRowCols;
  for (int t = tid; t < m * ng; t += kCT) {
    int i;
    const int j0 = small_div(t, m, i) * kRowCols;
    const double* a = q.Q + i * q.qrs;
    const double* b = Bs + 32 * j0;
    const int e = i - rho;  // row of R^-1 that E contributes, if any
    double acc[kRowCols];
#pragma unroll
    for (int c = 0; c < kRowCols; ++c) acc[c] = (e >= 0 && e < nc && j0 + c < nc) ? Ri[e + 33 * (j0 + c)] : 0.0;
#pragma unroll 8
    for (int k = 0; k < rho; ++k) {
      const double x = a[k * q.qcs];
#pragma unroll
      for (int c = 0; c < kRowCols; ++c) acc[c] = fma(x, b[k + 32 * c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < kRowCols; ++c)
      if (j0 + c < nc) C[i * q.qrs + (j0 + c) * q.qcs] = acc[c];
  }
  __syncthreads();
  return true;
}

__device__ __forceinline__ void wg_qr(const Qr& q) {
  const int m = q.m, n = q.n;
  if (q.rho == 1 && !q.R && m <= kRank1Rows) {
    rank1_qr(q);
    return;
  }
  if (q.rho >= 2 && q.rho <= kSmallRho && q.rho < n && !q.R && q.M != q.Q && (int64_t)m * q.rho <= kMsDoubles && n <= 256) {
    const bool done = small_capped_qr(q);
    __syncthreads();
    if (done) return;
  }
  if (q.rho >= n && m <= kQrRows && n <= 32 && cholqr2_reg(q)) return;
  // Tall (m > kQrRows, n <= 32): streamed CholeskyQR2.  A QR capped at
  // 2 <= rho < n proper reflectors (a local solution of rank at most rho, R not
  // wanted, M not Q) would make Householder stream the matrix through one CU
  // rho times; instead Q's first rho columns come from CholeskyQR2 of M's
  // first rho columns (Householder's, up to rounding, when those columns are
  // independent) and the other n - rho from orthonormalising the completion
  // e_j - Q_rho Q_rho(j,:)^T, j = rho..n-1 (identity reflectors give a
  // completion too; the update does not depend on which one).  A failed
  // Cholesky pivot leaves the decision to Householder, from M.
  if (m > kQrRows && n <= 32 && q.aux) {
    const bool capped = q.rho >= 2 && q.rho < n && !q.R && q.M != q.Q;
    if (q.rho >= n || capped) {
      bool ok = true;
      for (int pass = 0; pass < (capped ? 2 : 1) && ok; ++pass) {
        Qr a = q;
        if (capped && pass == 0) {
          a.n = q.rho;
          a.R = nullptr;
        } else if (capped) {
          if (capped_completion_closed(q)) break;
          capped_completion(q);
          a.n = n - q.rho;
          a.rho = a.n;
          a.M = q.Q + (int64_t)q.rho * q.qcs;
          a.mrs = q.qrs;
          a.mcs = q.qcs;
          a.Q = const_cast<double*>(a.M);
          a.R = nullptr;
        }
        ok = cholqr2_tall(a);
      }
      if (ok) return;
    }
  }
  if (m <= kQrRows && n <= 32) {
    // Householder in LDS
    const int mp = round16(m);
    const int ld = mp + 1;  // odd: walks across columns hit distinct banks
    __syncthreads();
    stage(kLdsMs, 1, ld, mp, 32, q.M, q.mrs, q.mcs, m, n);
    __syncthreads();
    householder_qr(q, s_lds + kLdsMs, ld);
    return;
  }
  // larger matrices: Householder in the device scratch buffer (a contiguous
  // column-major M is copied flat, eight loads in flight per thread)
  if (q.mrs == 1 && q.mcs == m) {
    const int64_t total = (int64_t)m * n;
#pragma unroll 8
    for (int64_t e = tix(); e < total; e += kCT) q.aux[e] = q.M[e];
  } else {
    for_each_ij(m, n, [&](int i, int j) { q.aux[i + (int64_t)m * j] = q.M[i * q.mrs + j * q.mcs]; });
  }
  __syncthreads();
  householder_qr(q, q.aux, m);
}

// ------------------------------------------------------------------ ops

__device__ __forceinline__ void exec_op(const ChainOp& op) {
  const int tid = tix();
  switch (op.type) {
    case kOpGemm:
      wg_gemm(Gemm{op.m, op.n, op.k, op.a, op.ars, op.acs, op.b, op.brs, op.bcs, op.c, op.crs, op.ccs, op.c32});
      break;
    case kOpQr:
      wg_qr(Qr{(int)op.m, (int)op.n, op.rho, op.a, op.ars, op.acs, op.c, op.crs, op.ccs, op.r, op.aux, op.tol});
      break;
    case kOpNormG: {
      // a = g in, c = g out (m = r_m); b = G_m in, r = G_m out (k elements)
      double p = 0.0;
      for (int i = tid; i < op.m; i += kCT) p = fma(op.a[i], op.a[i], p);
      const double nu = sqrt(block_sum(p, s_lds + kLdsRed));
      if (nu > 0.0) {
        const double inv = 1.0 / nu;
        for (int i = tid; i < op.m; i += kCT) op.c[i] = op.a[i] * inv;
#pragma unroll 8
        for (int64_t e = tid; e < op.k; e += kCT) op.r[e] = op.b[e] * nu;
      } else {
        for (int i = tid; i < op.m; i += kCT) op.c[i] = (i == 0) ? 1.0 : 0.0;
#pragma unroll 8
        for (int64_t e = tid; e < op.k; e += kCT) op.r[e] = op.b[e];
      }
      __syncthreads();
      break;
    }
    case kOpSpdInv: {
      // W = S + shift I (identity beyond m), R^-1 by chol_inv32, S^-1 = R^-1 R^-T
      const int n = (int)op.m;
      double* W = s_lds + kLdsW;
      double tr = 0.0;
      for (int i = 0; i < n; ++i) tr += op.a[i * op.ars + i * op.acs];
      const double shift = op.tol * tr / n;
      {
        const int i = tid & 31, j = tid >> 5;
        W[i + 32 * j] = (i < n && j < n) ? op.a[i * op.ars + j * op.acs] + (i == j ? shift : 0.0)
                                         : (i == j ? 1.0 : 0.0);
      }
      __syncthreads();
      const bool ok = chol_inv32<2>(s_lds + kLdsW, s_lds + kLdsR1, s_lds + kLdsRi, 0.0, n);
      if (!ok && tid == 0) *op.flag = 1;
      const View Riv{kLdsRi, 1, 33}, RiTv{kLdsRi, 33, 1};
      gemm_lds(n, n, 8, Riv, RiTv, [&](int ii, int jj, double v) { op.c[ii + n * jj] = v; });
      __syncthreads();
      break;
    }
    case kOpCopy:
#pragma unroll 8
      for (int64_t e = tid; e < op.m; e += kCT) {
        const double x = op.a[e];
        if (op.c) op.c[e] = x;
        if (op.c32) op.c32[e] = (float)x;
      }
      __syncthreads();
      break;
    case kOpCommit: {
      // a = new g (m = r_m); b = old state, c = new state (k doubles)
      const int f = *op.flag;
      const int64_t t = *op.tdev;
      if (f == 0) {
        if (op.hist && op.hist_cap > 0) {
          const int64_t row = t % op.hist_cap;
          for (int i = tid; i < op.m; i += kCT) op.hist[row * op.m + i] = op.a[i];
        }
      } else {
        for (int64_t e = tid; e < op.k; e += kCT) op.c[e] = op.b[e];
      }
      __syncthreads();
      if (tid == 0) {
        if (f == 0) *op.tdev = t + 1;
        else *op.rejected += 1;
        *op.flag = 0;
      }
      __syncthreads();
      break;
    }
    default:
      break;
  }
}

// Workgroup b runs the operations of segs[b]: one workgroup per stream of a
// batch (one stream alone: a batch of one).  The segments and operation lists
// are read-only while the kernel runs: reading them through the constant
// address space lets every operation descriptor arrive in scalar registers
// (through a generic pointer they would be fetched per lane and kept in vector
// registers, which spill).
typedef const TT_CONSTANT_AS ChainOp ConstChainOp;
typedef const TT_CONSTANT_AS ChainSeg ConstChainSeg;

__global__ void __launch_bounds__(kCT) k_chain(const ChainSeg* __restrict__ segs, int64_t* trace) {
  const ChainSeg sg = ((ConstChainSeg*)(const void*)segs)[blockIdx.x];
  ConstChainOp* ops = (ConstChainOp*)(uint64_t)sg.ops;
  const int count = sg.count;
  {
    // One burst of vector loads, one per 64-byte line of the segment's
    // descriptors, brings them into L2 together: each operation's scalar
    // descriptor load then waits for an L2 hit, not a trip to memory.
    const uint32_t* words = reinterpret_cast<const uint32_t*>(sg.ops);
    const int nw = count * (int)(sizeof(ChainOp) / 4);
    uint32_t acc = 0;
    for (int e = 16 * (int)threadIdx.x; e < nw; e += 16 * kCT) acc ^= words[e];
    asm volatile("" ::"v"(acc));
  }
  for (int i = 0; i < count; ++i) {
    const ChainOp op = ops[i];
    if (trace && threadIdx.x == 0) trace[2 * i] = (int64_t)wall_clock64();
    exec_op(op);
    __syncthreads();
    if (trace && threadIdx.x == 0) trace[2 * i + 1] = (int64_t)wall_clock64();
  }
}

__global__ void __launch_bounds__(kCT) k_chain_one(ChainOp op) { exec_op(op); }

constexpr size_t kChainLds = (size_t)kLdsTotal * sizeof(double);
bool g_chain_ready = false;

}  // namespace

hipError_t chain_setup(size_t lds_limit) {
  if (lds_limit < kChainLds) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)k_chain, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kChainLds);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_chain_one, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kChainLds);
  if (e != hipSuccess) return e;
  g_chain_ready = true;
  return hipSuccess;
}

bool chain_op_supported(const ChainOp& op) {
  if (op.type == kOpSpdInv) return op.m >= 1 && op.m <= 32;
  if (op.type == kOpQr) return op.n >= 1 && op.m >= op.n && op.n <= kMaxHouseholderCols && op.m <= INT32_MAX;
  if (op.type == kOpGemm) return op.m <= INT32_MAX && op.n <= INT32_MAX && op.k <= INT32_MAX;
  return true;
}

hipError_t chain_run(hipStream_t st, const ChainSeg* segs_dev, int nsegs, int64_t* trace) {
  if (nsegs == 0) return hipSuccess;
  if (!g_chain_ready) return hipErrorNotInitialized;
  if (nsegs < 0 || (trace && nsegs != 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chain, dim3(nsegs), dim3(kCT), kChainLds, st, segs_dev, trace);
  return hipGetLastError();
}

hipError_t chain_run_one(hipStream_t st, const ChainOp& op) {
  if (!g_chain_ready) return hipErrorNotInitialized;
  hipLaunchKernelGGL(k_chain_one, dim3(1), dim3(kCT), kChainLds, st, op);
  return hipGetLastError();
}

}  // namespace ttk
