// Internal declarations shared by the runtime and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstdint>

#include "tt_stream.h"

namespace ttk {

// Records `msg` as the calling thread's last error and returns `st`.
tt_status set_error(tt_status st, const char* msg);

// Device data that no thread writes while a kernel runs, reached through a
// pointer: in the device pass it is read through the constant address space,
// so uniform reads (operation descriptors) go to scalar registers.  The host
// pass never dereferences such pointers.
#if defined(__HIP_DEVICE_COMPILE__)
#define TT_CONSTANT_AS __attribute__((address_space(4)))
#else
#define TT_CONSTANT_AS
#endif
// Device memory reached through a pointer that the compiler cannot trace to a
// kernel argument (batch descriptors): loads through the global address space
// are plain vector-memory loads, where a generic pointer would give flat loads
// that also count against the LDS wait counter and force coarser waits.
#if defined(__HIP_DEVICE_COMPILE__)
#define TT_GLOBAL_AS __attribute__((address_space(1)))
#else
#define TT_GLOBAL_AS
#endif

// Threads of the workgroup that runs the chain operation lists.
constexpr int kChainThreads = 1024;

// ---------------------------------------------------------------- chain lists
// One operation of the update's FP64 chain, executed by the one-workgroup
// kernel of chain_exec.hip.  Field use by type:
//   kOpGemm   C(i,j) = sum_k A(i,k) B(k,j): m = rows, n = cols, k = depth;
//             a/ars/acs, b/brs/bcs, c/crs/ccs element strides; c may be null
//             when c32 (same strides) receives an FP32 copy; rho = kWideJb4
//             (below) marks a whole-GPU product for four outputs per thread.
//   kOpQr     thin QR of the m x n matrix a (strides ars, acs) into Q = c
//             (strides crs, ccs) and, if r != null, R (n x n column-major);
//             aux holds m*n doubles; rho = cap on proper reflectors; tol = rank
//             threshold relative to ||M||_F.  a may alias c.
//   kOpNormG  a = g in, c = g out (m = r_m); b = G_m in, r = G_m out (k values).
//   kOpCopy   c[e] = a[e] and/or c32[e] = (float)a[e], e < m.
//   kOpCommit if *flag == 0: hist row (t mod hist_cap) = a (m values), t += 1;
//             else c = b (k doubles, restoring the old state), *rejected += 1;
//             then *flag = 0.
//   kOpSpdInv c = (S + tol tr(S)/m I)^-1 for the symmetric m x m matrix a
//             (strides ars, acs; m <= 32), c column-major with leading
//             dimension m; a non-positive Cholesky pivot sets *flag = 1.
enum : int32_t { kOpGemm = 1, kOpQr = 2, kOpNormG = 3, kOpCopy = 4, kOpCommit = 5, kOpSpdInv = 6 };
struct ChainOp {
  int32_t type = 0;
  int32_t rho = 0;
  int64_t m = 0, n = 0, k = 0;
  const double* a = nullptr;
  int64_t ars = 0, acs = 0;
  const double* b = nullptr;
  int64_t brs = 0, bcs = 0;
  double* c = nullptr;
  int64_t crs = 0, ccs = 0;
  float* c32 = nullptr;
  double* r = nullptr;
  double* aux = nullptr;
  double tol = 0.0;
  int* flag = nullptr;
  int* rejected = nullptr;
  int64_t* tdev = nullptr;
  double* hist = nullptr;
  int64_t hist_cap = 0;
};
// Sets the kernels' LDS size; once per process before the first launch.
hipError_t chain_setup(size_t lds_limit);
bool chain_op_supported(const ChainOp& op);
// A run of consecutive operations of one stream's list.
struct ChainSeg {
  const ChainOp* ops;
  int32_t count;
  int32_t pad;
};
// Workgroup b runs segs[b] (device array of nsegs segments; a segment may be
// empty).  If trace is not null (nsegs == 1 only), trace[2i] and trace[2i+1]
// receive the device wall clock at the start and end of operation i.
hipError_t chain_run(hipStream_t st, const ChainSeg* segs_dev, int nsegs, int64_t* trace = nullptr);
// Runs one operation passed by value.
hipError_t chain_run_one(hipStream_t st, const ChainOp& op);
// Rows of the slice staged per wave in pass 2 (multiple of 8).
constexpr int kPass2SlabMax = 72;
constexpr int kPass2Waves = 8;

// ---------------------------------------------------------------- chain (FP64)
// C(i,j) = sum_k A(i,k) B(k,j) over the whole GPU, element strides; C may be
// null when C32 (same strides) receives an FP32 copy.
hipError_t gemm64(hipStream_t st, int64_t M, int64_t N, int64_t K,
                  const double* A, int64_t ars, int64_t acs,
                  const double* B, int64_t brs, int64_t bcs,
                  double* C, int64_t crs, int64_t ccs, float* C32);

// The GEMMs *ops[b] (kOpGemm; device array of nops op pointers, shapes may
// differ) over the whole GPU, grid (gx, nops); gx must cover the largest
// (gemm64_blocks).  Each product's split of the depth depends on its own shape
// only, so a product computes the same bits in any batch.
// A whole-GPU product whose ChainOp has rho == kWideJb4 computes four
// consecutive output columns per thread where its layout allows (plans for
// batched waves mark their large products so); the result is the same bits.
constexpr int32_t kWideJb4 = 4;
int64_t gemm64_blocks(int64_t M, int64_t N, int64_t K, int64_t ars, int64_t acs, int64_t brs, int64_t bcs,
                      bool jb4);
hipError_t gemm64_ops(hipStream_t st, const ChainOp* const* ops_dev, int nops, int64_t gx);

// Element conversion FP64 -> out dtype (F64/F32).
hipError_t convert_out(hipStream_t st, const double* src, void* dst, tt_dtype dt, int64_t n);

// ---------------------------------------------------------------- passes (FP32)
// Pass 1: Z(p,a) = sum_j X(p,j) B(a,j), X P x J (p fastest) of dtype `xdt`,
// B r x J FP32; Z written FP64 (P x r column-major) from FP32 partial tiles
// (ws, plan.ws_floats floats) added in FP64.  Sets *flag if Z is non-finite.
// One member of a batched pass launch: the slice x (the batch's element
// type), the interface w (B for pass 1, A for pass 2), the output (Z or Y),
// the pass's workspace (FP32 partial tiles), the non-finite flag, the
// member's P, J, r and its plan's tiles and chunks.  Members of one launch
// share the kernel's template shape (rows per lane, waves, rank tiles).
struct PassDesc {
  const void* x;
  const float* w;
  double* out;
  float* ws;
  int* flag;
  int64_t P, J;
  int32_t r, tiles, chunks, pad;
};
// A batched pass launch: n members (device array), grid.x of the main and
// the reduction kernel covering the largest member (blocks past a member's
// own grid return at once).
struct PassLaunch {
  const PassDesc* desc;
  int n;
  unsigned gx, grx;
};

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
// With bl != null the grid gains a member index and every member's pointers,
// shape and tiles come from bl->desc (X, P, J, r, B, Z, ws, flag and the
// plan's tiles and chunks are then ignored; the plan's template shape must be
// every member's).  pass1_grids gives the main and reduction grid.x of a
// member.
hipError_t pass1(hipStream_t st, const void* X, tt_dtype xdt, const Pass1Plan& plan, int64_t P, int64_t J, int r,
                 const float* B, double* Z, float* ws, int* flag, const PassLaunch* bl = nullptr);
void pass1_grids(const Pass1Plan& plan, int64_t P, unsigned* gx, unsigned* grx);

// When set (not null), the pass launchers record this event on their stream
// right after a pass's contraction kernel, before its partial-tile reduction
// (or after the only kernel), so the contraction kernel can be timed alone.
// Per calling thread; the runtime sets it around one pass and clears it.
hipEvent_t& pass_mid_event();
// Which kernels the pass launchers launch: bit 0 the contraction kernel, bit
// 1 the partial-tile reduction (default 3).  Per calling thread; only the
// pass timer changes it (to launch either kernel alone, back to back).
int& pass_launch_mask();

// Pass 2: Y(a,j) = sum_p A(p,a) X(p,j); A P x r FP32 column-major; Y FP64
// r x J column-major.  Sets *flag if Y non-finite.
hipError_t pass2(hipStream_t st, const void* X, tt_dtype xdt, int64_t P, int64_t J, int r,
                 const float* A, double* Y, int* flag, const PassLaunch* bl = nullptr);
unsigned pass2_grid(int64_t J);
// Template shape of pass 2 for these sizes (members of one launch share it).
int pass2_vec(int64_t P);
// Whether pass 2 runs the grouped FP32 kernel k_pass2g for these sizes (FP32
// slices, 4 <= P <= 1280, r <= 32; when P % 4 != 0 also P J < 2^30), and
// its waves per column tile (1, 2, 4, 8 or 16, from P); both are part of the template shape too.  Its batched grid
// is pass2_grid(J) like k_pass2's (blocks past a member's tiles return).
bool pass2_grouped(int64_t P, int64_t J, int r, tt_dtype xdt);
int pass2g_nwt(int64_t P);

// ---------------------------------------------------------------- passes (BF16)
// The same two contractions with the slice and the interface rounded to BF16
// (round to nearest even) and FP32 accumulation (v_mfma_f32_32x32x16_bf16).
// Blocks that split a tile's reduction write FP32 partial tiles to the
// workspace (no initialisation needed), added in FP64 in chunk order by a
// second kernel; a block that covers the whole reduction writes the result.
struct PassBPlan {
  int vec = 1;        // pass 1: rows per lane (row tile = 32 vec); 8, 4 or 1
  int waves = 4;      // waves per block
  int tiles = 1;      // pass 1: row tiles; pass 2: 32-column tiles
  int chunks = 1;     // pass 1: column-group chunks; pass 2: row chunks
  int ntn = 1;        // 32-column tiles of the rank
  int staged = 0;     // pass 2: the LDS-staged kernel (P % 8 == 0; one chunk, no workspace use)
  size_t ws_bytes = 0;
};
PassBPlan pass1b_plan(int64_t P, int64_t J, int r, int cus);
PassBPlan pass2b_plan(int64_t P, int64_t J, int r, int cus);
// Recomputes tiles and ws_bytes after the tunable fields were set.
PassBPlan pass1b_finish(PassBPlan pl, int64_t P, int64_t J);
PassBPlan pass2b_finish(PassBPlan pl, int64_t P, int64_t J);
hipError_t pass1_bf16(hipStream_t st, const void* X, tt_dtype xdt, const PassBPlan& plan, int64_t P, int64_t J,
                      int r, const float* B, double* Z, void* ws, int* flag, const PassLaunch* bl = nullptr);
hipError_t pass2_bf16(hipStream_t st, const void* X, tt_dtype xdt, const PassBPlan& plan, int64_t P, int64_t J,
                      int r, const float* A, double* Y, void* ws, int* flag, const PassLaunch* bl = nullptr);
void pass1b_grids(const PassBPlan& plan, unsigned* gx, unsigned* grx);
void pass2b_grids(const PassBPlan& plan, unsigned* gx, unsigned* grx);
// Pass 2 (BF16) loads 8-row vectors when P % 8 == 0 (part of its template
// shape: members of one launch share it).
bool pass2b_vx(int64_t P);
// Dynamic LDS limits of the BF16 kernels (the staged pass 2 needs 76 KB);
// once per process before their first launch, like pass_setup.
hipError_t pass_bf16_setup();

// ---------------------------------------------------------------- tuner
struct PassPlans {
  Pass1Plan p1;           // FP32 contractions
  PassBPlan p1b, p2b;     // BF16 contractions
  bool tuned = false;
  float ms = 0.f;         // tuned: device time of pass 1 + pass 2 with these plans
};
PassPlans default_pass_plans(int64_t P, int64_t J, int r, int cus);
// Plans of the fastest measured launch shapes for (P, J, r) and the given
// contraction precision, timed on stream st (synchronised) the first time a
// shape is seen in the process and cached afterwards.
hipError_t tuned_pass_plans(int64_t P, int64_t J, int r, tt_dtype compute, int cus, hipStream_t st,
                            PassPlans* out);

// Reconstruction of the latest slice: out = G_1 x ... x G_m x g (FP64 chain).
// Implemented on the runtime side with gemm64.

}  // namespace ttk
