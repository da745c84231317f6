// Host runtime of the C ABI declared in include/tt_stream.h.
//
// One handle holds one stream's state on one GPU: two FP64 state buffers
// (cores G_1..G_m then the temporal vector g) used in turn, the committed one
// being state[cur], plus the workspace of one update.  An update (Algorithm 1)
// is planned once, at creation, for each of the two parities:
//   right-orthogonalisation   normalise g, LQ sweep k = m..2 (Section 3.4.1)
//   right interfaces          B_k = G_{k+1} x_3 B_{k+1}, k = m-1..k*
//   pass 1                    Z = X^<k*> B_{k*}^T          (slice stream)
//   head                      Z_k for k < k*; for k = 1..k*: G~_k = A_k^T Z_k,
//                             thin QR, A_{k+1} = A_k x G_k  (Eq. 5 reassociated)
//   pass 2                    Y = A_{k*+1}^T X^<k*>          (slice stream)
//   tail                      for k = k*+1..m: G~_k = Y_k B_k^T, thin QR,
//                             Y_{k+1} = G_k^T Y_k; g = Y_{m+1}
//   commit                    history row and t, or restore of the old state
//                             when the slice was not finite
// The new state is written to state[cur ^ 1]; the host flips cur after
// enqueueing.  Small steps are grouped into operation lists run by one
// workgroup (chain_exec.hip); large contractions and the passes are launches
// of their own.  Nothing is read back to the host during a push.
#include "stream_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <array>
#include <unordered_map>
#include <vector>

namespace ttk {
hipError_t pass_setup();
}  // namespace ttk

using ttk::Step;
using ttk::UpdatePlan;
using ttk::kStepChain;
using ttk::kStepWide;
using ttk::kStepPass1;
using ttk::kStepPass2;
using ttk::kStepMark;

namespace {

constexpr uint64_t kDead = 0xdeadbeefdeadbeefULL;
constexpr double kQrTol = 64.0 * 2.220446049250313e-16;
// A contraction of at least kWideFma multiply-adds, or a deep one (depth at
// least kWideDepth and kWideDeepFma multiply-adds: a long dot product per
// output, bound by one workgroup's load latency), is launched over the whole
// GPU instead of being run by the chain workgroup.  On MI355X a whole-GPU
// launch costs about 5-6 us plus a few us where it splits the chain, while
// the chain workgroup takes 20-35 us for products of 0.5-0.7 M multiply-adds
// (staging and writing them through one CU), hence these thresholds.
constexpr double kWideFma = 2.0e5;
constexpr double kWideFmaWave = 4.0e5;  // with TT_FLAG_WAVE_PLAN
constexpr double kWideJb4Fma = 4.0e6;   // with TT_FLAG_WAVE_PLAN: blocked whole-GPU products from this size
constexpr int64_t kWideDepth = 256;
constexpr double kWideDeepFma = 3.0e4;

thread_local std::string g_last_error = "no error";

tt_status fail(tt_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define TT_HIP(call)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail(TT_ERR_DEVICE, std::string(#call) + " failed: " + hipGetErrorString(e_));     \
  } while (0)

size_t dtype_size(tt_dtype d) { return d == TT_F64 ? 8 : d == TT_F32 ? 4 : 2; }

bool mul_ok(int64_t a, int64_t b, int64_t* out) {
  if (a <= 0 || b <= 0) return false;
  if (a > INT64_MAX / b) return false;
  *out = a * b;
  return true;
}

// SplitMix64 (Steele, Lea, Flood 2014) and the Box-Muller transform give the
// optional seeded N(0,1) initial cores.
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

void normal_fill(std::vector<double>& v, uint64_t seed) {
  uint64_t s = seed;
  const double two_pi = 6.283185307179586476925286766559;
  for (size_t i = 0; i < v.size(); i += 2) {
    double u1 = ((splitmix64(s) >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0,1]
    double u2 = (splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
    double rad = std::sqrt(-2.0 * std::log(u1));
    v[i] = rad * std::cos(two_pi * u2);
    if (i + 1 < v.size()) v[i + 1] = rad * std::sin(two_pi * u2);
  }
}

}  // namespace

tt_status ttk::set_error(tt_status st, const char* msg) { return fail(st, msg); }

namespace {
std::mutex g_handles_mu;
std::unordered_map<const void*, int>& live_handles() {
  static std::unordered_map<const void*, int> m;
  return m;
}
}  // namespace

void ttk::handle_register(const void* p, int kind) {
  std::lock_guard<std::mutex> lk(g_handles_mu);
  live_handles()[p] = kind;
}

void ttk::handle_unregister(const void* p) {
  std::lock_guard<std::mutex> lk(g_handles_mu);
  live_handles().erase(p);
}

bool ttk::handle_live(const void* p, int kind) {
  std::lock_guard<std::mutex> lk(g_handles_mu);
  const auto it = live_handles().find(p);
  return it != live_handles().end() && it->second == kind;
}

hipError_t ttk::stream_quiesce(const tt_stream* s) {
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess && s->ext_done) e = hipEventSynchronize(s->ext_done);
  return e;
}


namespace {

bool valid(const tt_stream* s) { return ttk::stream_valid(s); }

void* dev_alloc(tt_stream* s, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (s->has_alloc) {
    p = s->alloc.alloc(bytes, s->alloc.ctx);
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();  // the failure is reported as OOM; it must not resurface at a later launch check
    }
  }
  if (p) {
    s->owned.push_back(p);
    s->device_bytes += bytes;
  }
  return p;
}

void release(tt_stream* s) {
  for (void* p : s->owned) {
    if (s->has_alloc) s->alloc.free(p, s->alloc.ctx);
    else (void)hipFree(p);
  }
  s->owned.clear();
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->evcopy) (void)hipEventDestroy(s->evcopy);
  if (s->evcommit) (void)hipEventDestroy(s->evcommit);
  for (hipEvent_t& e : s->evpass)
    if (e) (void)hipEventDestroy(e);
}

tt_status check_shape(int32_t m, const int64_t* modes, const int64_t* ranks) {
  if (m < 1) return fail(TT_ERR_SHAPE, "n_slice_modes must be >= 1");
  int64_t N = 1;
  for (int k = 0; k < m; ++k) {
    if (modes[k] < 1) return fail(TT_ERR_SHAPE, "mode sizes must be >= 1");
    if (!mul_ok(N, modes[k], &N) || N > (int64_t(1) << 40)) return fail(TT_ERR_SHAPE, "slice size overflows");
    if (ranks && ranks[k] < 1) return fail(TT_ERR_SHAPE, "ranks must be >= 1");
  }
  return TT_OK;
}

void clamp(int32_t m, const int64_t* modes, const int64_t* in, int64_t* out) {
  std::vector<int64_t> r(m + 1);
  r[0] = 1;
  for (int k = 1; k <= m; ++k) r[k] = in[k - 1];
  for (int k = 1; k <= m; ++k) {
    int64_t cap;
    if (!mul_ok(r[k - 1], modes[k - 1], &cap)) cap = INT64_MAX;
    if (r[k] > cap) r[k] = cap;
  }
  for (int k = m; k >= 2; --k) {
    int64_t cap;
    if (!mul_ok(modes[k - 1], r[k], &cap)) cap = INT64_MAX;
    if (r[k - 1] > cap) r[k - 1] = cap;
  }
  for (int k = 1; k <= m; ++k) out[k - 1] = r[k];
}

// Split point: the k in [1, m] that minimises the size of the two pass
// outputs, P_k r_k + J_k r_k (pass 1 writes P_k x r_k, pass 2 writes
// r_k x J_k, and the chain work on each side scales with them).
int choose_split(const tt_stream* s) {
  int best = 1;
  double bestc = 1e300;
  for (int k = 1; k <= s->m; ++k) {
    if (s->r[k] > 64) continue;
    const double c = (double)s->Pk[k] * s->r[k] + (double)s->Jk[k] * s->r[k];
    if (c < bestc) {
      bestc = c;
      best = k;
    }
  }
  return best;
}

// Split point with TT_FLAG_AUTOTUNE: the split points whose modelled pass
// output (P_k + J_k) r_k is within a factor 4 of the smallest (at most three,
// in model order) are timed with their tuned pass plans, and the one with the
// fastest pair of passes wins (ties: the earlier in model order).  The pass
// times are cached per shape, so the choice repeats within a process and
// every stream of one shape gets the same split point.
bool tune_split(tt_stream* s, int cus) {
  std::vector<std::pair<double, int>> cand;
  for (int k = 1; k <= s->m; ++k)
    if (s->r[k] <= 64) cand.push_back({(double)(s->Pk[k] + s->Jk[k]) * (double)s->r[k], k});
  if (cand.empty()) return true;
  std::stable_sort(cand.begin(), cand.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  float best = 0.f;
  int bestk = -1, tried = 0;
  for (const auto& [cost, k] : cand) {
    if (tried == 3 || cost > 4.0 * cand[0].first) break;
    ++tried;
    ttk::PassPlans pl;
    if (ttk::tuned_pass_plans(s->Pk[k], s->Jk[k], (int)s->r[k], s->compute, cus, s->stream, &pl) != hipSuccess)
      return false;
    if (bestk < 0 || pl.ms < best) {
      best = pl.ms;
      bestk = k;
    }
  }
  if (bestk > 0) s->kstar = bestk;
  return true;
}

void plan_chain(UpdatePlan& p, const ttk::ChainOp& op) {
  p.ops.push_back(op);
  const int idx = (int)p.ops.size() - 1;
  if (!p.steps.empty() && p.steps.back().kind == kStepChain && p.steps.back().first + p.steps.back().count == idx)
    p.steps.back().count++;
  else
    p.steps.push_back({kStepChain, idx, 1});
}

// Byte range [lo, hi) an m x n operand with element strides rs, cs spans.
struct Span {
  uintptr_t lo = 0, hi = 0;
};
Span span_of(const void* p, int64_t m, int64_t n, int64_t rs, int64_t cs, size_t elem) {
  Span r;
  if (!p || m <= 0 || n <= 0) return r;
  r.lo = reinterpret_cast<uintptr_t>(p);
  r.hi = r.lo + (size_t)((m - 1) * rs + (n - 1) * cs + 1) * elem;
  return r;
}
bool overlap(const Span& a, const Span& b) { return a.lo < b.hi && b.lo < a.hi; }

// True if product y neither reads nor writes what product x writes, nor
// writes what x reads: the two may run in one launch.
bool independent(const ttk::ChainOp& x, const ttk::ChainOp& y) {
  const Span xw[2] = {span_of(x.c, x.m, x.n, x.crs, x.ccs, 8), span_of(x.c32, x.m, x.n, x.crs, x.ccs, 4)};
  const Span xr[2] = {span_of(x.a, x.m, x.k, x.ars, x.acs, 8), span_of(x.b, x.k, x.n, x.brs, x.bcs, 8)};
  const Span yw[2] = {span_of(y.c, y.m, y.n, y.crs, y.ccs, 8), span_of(y.c32, y.m, y.n, y.crs, y.ccs, 4)};
  const Span yr[2] = {span_of(y.a, y.m, y.k, y.ars, y.acs, 8), span_of(y.b, y.k, y.n, y.brs, y.bcs, 8)};
  for (const Span& w : xw)
    for (const Span& r : yr)
      if (overlap(w, r)) return false;
  for (const Span& w : yw) {
    for (const Span& r : xr)
      if (overlap(w, r)) return false;
    for (const Span& v : xw)
      if (overlap(w, v)) return false;
  }
  return true;
}

// C = A B (see ttk::ChainOp); large products become launches of their own,
// and a large product independent of the large products planned right
// before it joins their launch.
double wide_fma_of(const tt_stream* s) { return (s->flags & TT_FLAG_WAVE_PLAN) ? kWideFmaWave : kWideFma; }

void plan_gemm(UpdatePlan& p, int64_t M, int64_t N, int64_t K, const double* A, int64_t ars, int64_t acs,
               const double* B, int64_t brs, int64_t bcs, double* C, int64_t crs, int64_t ccs, float* C32) {
  ttk::ChainOp op;
  op.type = ttk::kOpGemm;
  op.m = M;
  op.n = N;
  op.k = K;
  op.a = A;
  op.ars = ars;
  op.acs = acs;
  op.b = B;
  op.brs = brs;
  op.bcs = bcs;
  op.c = C;
  op.crs = crs;
  op.ccs = ccs;
  op.c32 = C32;
  const double fma = (double)M * (double)N * (double)K;
  if (fma >= p.wide_fma || (K >= kWideDepth && fma >= kWideDeepFma)) {
    // plans for batched waves: large products take four outputs per thread
    if (p.wide_fma > kWideFma && fma >= kWideJb4Fma) op.rho = ttk::kWideJb4;
    p.ops.push_back(op);
    const int idx = (int)p.ops.size() - 1;
    bool join = !p.steps.empty() && p.steps.back().kind == kStepWide &&
                p.steps.back().first + p.steps.back().count == idx;
    for (int q = join ? p.steps.back().first : idx; join && q < idx; ++q) join = independent(p.ops[q], op);
    if (join)
      p.steps.back().count++;
    else
      p.steps.push_back({kStepWide, idx, 1});
  } else {
    plan_chain(p, op);
  }
}

// Thin QR of the m x n matrix M into Q (strides as in ttk::ChainOp).
void plan_qr(UpdatePlan& p, const tt_stream* s, int64_t m, int64_t n, int rho, const double* M, int64_t mrs,
             int64_t mcs, double* Q, int64_t qrs, int64_t qcs, double* R) {
  ttk::ChainOp op;
  op.type = ttk::kOpQr;
  op.m = m;
  op.n = n;
  op.rho = rho;
  op.a = M;
  op.ars = mrs;
  op.acs = mcs;
  op.c = Q;
  op.crs = qrs;
  op.ccs = qcs;
  op.r = R;
  op.aux = s->qrwork;
  op.tol = kQrTol;
  plan_chain(p, op);
}

void plan_copy(UpdatePlan& p, const double* src, double* dst, float* dst32, int64_t n) {
  ttk::ChainOp op;
  op.type = ttk::kOpCopy;
  op.m = n;
  op.a = src;
  op.c = dst;
  op.c32 = dst32;
  plan_chain(p, op);
}

// S^-1 of the symmetric positive definite m x m matrix S into Sinv.
void plan_spd_inv(UpdatePlan& p, const tt_stream* s, int64_t m, const double* S, double* Sinv) {
  ttk::ChainOp op;
  op.type = ttk::kOpSpdInv;
  op.m = m;
  op.a = S;
  op.ars = 1;
  op.acs = m;
  op.c = Sinv;
  op.tol = 0.0;
  op.flag = s->flag;
  plan_chain(p, op);
}

// The "w/o Ortho" ablation (TT_FLAG_NO_ORTHO): the update without the
// right-orthogonalisation (no normalisation of g, no LQ sweep).  The right
// interfaces B_k built from the current cores are then not orthonormal, and
// the exact local solution needs their Gram matrix:
//   G~_k = A_k^T X B_k^T R_k,  R_k = (B_k B_k^T)^+,
// R_k = (B_k B_k^T)^-1 when r_k <= J_k, else B_k (B_k^T B_k)^-2 B_k^T (B_k of
// full column rank; always the case at k = m, B_m = g).  The forward sweep's
// QR and everything after it are as in build_plan.  For k < k* the Gram
// matrix comes from the recursion B_k B_k^T = sum_i G_{k+1}(:,i,:)
// (B_{k+1} B_{k+1}^T) G_{k+1}(:,i,:)^T and needs r_k <= J_k.
void build_plan_noortho(tt_stream* s, int par) {
  UpdatePlan& P = s->plan[par];
  P.ops.clear();
  P.wide_fma = wide_fma_of(s);
  P.steps.clear();
  double* master = s->state[par];
  double* fresh = s->state[par ^ 1];
  double* tmp = s->gram_tmp;
  const int m = s->m, ks = s->kstar;
  const auto& I = s->I;
  const auto& r = s->r;
  const auto& Pk = s->Pk;
  const auto& Jk = s->Jk;
  auto Bk = [&](int k) -> double* { return k == m ? s->g_of(master) : s->B[k]; };

  // right interfaces B_{m-1} .. B_{k*} from the current cores
  for (int j = m - 1; j >= ks; --j) {
    const int64_t rj = r[j] * I[j + 1];
    plan_gemm(P, rj, Jk[j + 1], r[j + 1], s->G_of(master, j + 1), 1, rj, Bk(j + 1), 1, r[j + 1], s->B[j], 1, rj,
              j == ks ? s->B32 : nullptr);
  }
  if (ks == m) plan_copy(P, s->g_of(master), nullptr, s->B32, r[m]);
  // R_k for k >= k* from the explicit interfaces
  for (int k = m; k >= ks; --k) {
    const double* Bm = Bk(k);
    const int64_t rk = r[k], J = Jk[k];
    if (rk <= J) {
      plan_gemm(P, rk, rk, J, Bm, 1, rk, Bm, rk, 1, s->GB[k], 1, rk, nullptr);
      plan_spd_inv(P, s, rk, s->GB[k], s->GBi[k]);
    } else {
      // (B B^T)^+ = B H H B^T with H = (B^T B)^-1 (J x J)
      plan_gemm(P, J, J, rk, Bm, rk, 1, Bm, 1, rk, s->gram_j, 1, J, nullptr);
      plan_spd_inv(P, s, J, s->gram_j, s->gram_ji);
      plan_gemm(P, rk, J, J, Bm, 1, rk, s->gram_ji, 1, J, tmp, 1, rk, nullptr);
      plan_gemm(P, rk, J, J, tmp, 1, rk, s->gram_ji, 1, J, tmp + rk * J, 1, rk, nullptr);
      plan_gemm(P, rk, rk, J, tmp + rk * J, 1, rk, Bm, rk, 1, s->GBi[k], 1, rk, nullptr);
    }
  }
  // R_k for k < k* by the Gram recursion from B_{k*} B_{k*}^T
  if (ks > 1) {
    if (r[ks] > Jk[ks]) plan_gemm(P, r[ks], r[ks], Jk[ks], Bk(ks), 1, r[ks], Bk(ks), r[ks], 1, s->GB[ks], 1, r[ks],
                                  nullptr);
    for (int k = ks - 1; k >= 1; --k) {
      const int64_t rows = r[k] * I[k + 1];
      const double* G = s->G_of(master, k + 1);
      plan_gemm(P, rows, r[k + 1], r[k + 1], G, 1, rows, s->GB[k + 1], 1, r[k + 1], tmp, 1, rows, nullptr);
      plan_gemm(P, r[k], r[k], I[k + 1] * r[k + 1], tmp, 1, r[k], G, r[k], 1, s->GB[k], 1, r[k], nullptr);
      plan_spd_inv(P, s, r[k], s->GB[k], s->GBi[k]);
    }
  }

  P.steps.push_back({kStepPass1, 0, 0});

  auto Zof = [&](int k) -> double* { return k == ks ? s->Z : s->Zk[k]; };
  for (int k = ks - 1; k >= 1; --k) {
    const int64_t Kd = I[k + 1] * r[k + 1];
    plan_gemm(P, Pk[k], r[k], Kd, Zof(k + 1), 1, Pk[k], s->G_of(master, k + 1), r[k], 1, Zof(k), 1, Pk[k],
              nullptr);
  }
  // G~ R_k (rows x n) into gram_g, then the thin QR into the fresh core
  auto solve_qr = [&](int k, const double* src) {
    const int64_t rows = r[k - 1] * I[k];
    const int64_t n = r[k];
    plan_gemm(P, rows, n, n, src, 1, rows, s->GBi[k], 1, n, s->gram_g, 1, rows, nullptr);
    double* Gnew = s->G_of(fresh, k);
    plan_qr(P, s, rows, n, (int)std::min<int64_t>(n, Jk[k]), s->gram_g, 1, rows, Gnew, 1, rows, nullptr);
    return Gnew;
  };
  for (int k = 1; k <= ks; ++k) {
    const double* Gt;
    if (k == 1) {
      Gt = Zof(1);
    } else {
      const double* Ak = (k == 2) ? s->G_of(fresh, 1) : s->A[k];
      plan_gemm(P, r[k - 1], I[k] * r[k], Pk[k - 1], Ak, Pk[k - 1], 1, Zof(k), 1, Pk[k - 1], s->Gt, 1, r[k - 1],
                nullptr);
      Gt = s->Gt;
    }
    double* Gnew = solve_qr(k, Gt);
    if (k >= 2) {
      const double* Ak = (k == 2) ? s->G_of(fresh, 1) : s->A[k];
      double* Anext = (k == ks) ? nullptr : s->A[k + 1];
      plan_gemm(P, Pk[k - 1], I[k] * r[k], r[k - 1], Ak, 1, Pk[k - 1], Gnew, 1, r[k - 1], Anext, 1, Pk[k - 1],
                k == ks ? s->A32 : nullptr);
    } else if (ks == 1) {
      plan_copy(P, Gnew, nullptr, s->A32, Pk[1] * r[1]);
    }
  }

  P.steps.push_back({kStepPass2, 0, 0});

  int cur = 0;
  for (int k = ks + 1; k <= m; ++k) {
    const int64_t rows = r[k - 1] * I[k];
    const int64_t n = r[k];
    plan_gemm(P, rows, n, Jk[k], s->Y[cur], 1, rows, Bk(k), r[k], 1, s->Gt, 1, rows, nullptr);
    double* Gnew = solve_qr(k, s->Gt);
    double* dst = (k == m) ? s->g_of(fresh) : s->Y[cur ^ 1];
    plan_gemm(P, n, Jk[k], rows, Gnew, rows, 1, s->Y[cur], 1, rows, dst, 1, n, nullptr);
    cur ^= 1;
  }
  if (ks == m) plan_copy(P, s->Y[0], s->g_of(fresh), nullptr, r[m]);

  {
    ttk::ChainOp op;
    op.type = ttk::kOpCommit;
    op.a = s->g_of(fresh);
    op.m = r[m];
    op.b = master;
    op.c = fresh;
    op.k = s->state_len;
    op.flag = s->flag;
    op.rejected = s->rejected;
    op.tdev = s->tdev;
    op.hist = s->hist;
    op.hist_cap = s->hist_cap;
    plan_chain(P, op);
  }
}

// The right-orthogonalisation of the state `master` (Algorithm 1, step 1:
// normalise g, LQ sweep k = m..2) into the work state, then the right
// interfaces B_k, k = m-1..k* (step 2), B_{k*} also in FP32 for pass 1.
// The committed state is only read.
void plan_sweep(tt_stream* s, UpdatePlan& P, double* master) {
  double* work = s->work;
  const int m = s->m, ks = s->kstar;
  const auto& I = s->I;
  const auto& r = s->r;
  const auto& Jk = s->Jk;
  {
    ttk::ChainOp op;
    op.type = ttk::kOpNormG;
    op.a = s->g_of(master);
    op.c = s->g_of(work);
    op.m = r[m];
    op.b = s->G_of(master, m);
    op.r = s->G_of(work, m);
    op.k = r[m - 1] * I[m] * r[m];
    plan_chain(P, op);
  }
  auto Bk = [&](int k) -> double* { return k == m ? s->g_of(work) : s->B[k]; };
  for (int k = m; k >= 2; --k) {
    const int64_t rows = I[k] * r[k];
    const int64_t n = r[k - 1];
    double* Gk = s->G_of(work, k);
    // LQ of the r_{k-1} x (I_k r_k) unfolding = QR of its transpose
    plan_qr(P, s, rows, n, (int)n, Gk, n, 1, Gk, n, 1, s->Rbuf);
    // G_{k-1} <- G_{k-1} x_3 L with L = R^T
    const int64_t rows2 = r[k - 2] * I[k - 1];
    plan_gemm(P, rows2, n, n, s->G_of(master, k - 1), 1, rows2, s->Rbuf, n, 1, s->G_of(work, k - 1), 1, rows2,
              nullptr);
    // right interface B_{k-1} = G_k x_3 B_k, once G_k is final (B_{k*} after the sweep)
    if (k - 1 > ks) {
      const int j = k - 1;
      const int64_t rj = r[j] * I[j + 1];
      plan_gemm(P, rj, Jk[j + 1], r[j + 1], s->G_of(work, j + 1), 1, rj, Bk(j + 1), 1, r[j + 1], s->B[j], 1, rj,
                nullptr);
    }
  }
  if (ks < m) {
    const int64_t rj = r[ks] * I[ks + 1];
    plan_gemm(P, rj, Jk[ks + 1], r[ks + 1], s->G_of(work, ks + 1), 1, rj, Bk(ks + 1), 1, r[ks + 1], nullptr, 1, rj,
              s->B32);
  } else {
    plan_copy(P, s->g_of(work), nullptr, s->B32, r[m]);
  }
}

// The update that reads state[par] and writes state[par ^ 1].  Its steps 1-2
// (the right-orthogonalisation and the right interfaces) read only the
// committed state, so they are planned at the end of the previous update,
// right after its commit (plan_sweep of the state just committed; the first
// update's is run at creation and after set_state): an update starts with
// pass 1, and its commit is not delayed by the next update's sweep.
void build_plan(tt_stream* s, int par) {
  UpdatePlan& P = s->plan[par];
  P.ops.clear();
  P.wide_fma = wide_fma_of(s);
  P.steps.clear();
  double* master = s->state[par];
  double* fresh = s->state[par ^ 1];
  double* work = s->work;
  const int m = s->m, ks = s->kstar;
  const auto& I = s->I;
  const auto& r = s->r;
  const auto& Pk = s->Pk;
  const auto& Jk = s->Jk;
  auto Bk = [&](int k) -> double* { return k == m ? s->g_of(work) : s->B[k]; };

  P.steps.push_back({kStepPass1, 0, 0});

  // head: Z_k for k < k* from the right-orthogonal cores
  auto Zof = [&](int k) -> double* { return k == ks ? s->Z : s->Zk[k]; };
  for (int k = ks - 1; k >= 1; --k) {
    const int64_t Kd = I[k + 1] * r[k + 1];
    plan_gemm(P, Pk[k], r[k], Kd, Zof(k + 1), 1, Pk[k], s->G_of(work, k + 1), r[k], 1, Zof(k), 1, Pk[k], nullptr);
  }
  // forward sweep k = 1..k*
  for (int k = 1; k <= ks; ++k) {
    const int64_t rows = r[k - 1] * I[k];
    const int64_t n = r[k];
    const double* Gt;
    if (k == 1) {
      Gt = Zof(1);
    } else {
      const double* Ak = (k == 2) ? s->G_of(fresh, 1) : s->A[k];
      plan_gemm(P, r[k - 1], I[k] * r[k], Pk[k - 1], Ak, Pk[k - 1], 1, Zof(k), 1, Pk[k - 1], s->Gt, 1, r[k - 1],
                nullptr);
      Gt = s->Gt;
    }
    double* Gnew = s->G_of(fresh, k);
    plan_qr(P, s, rows, n, (int)std::min<int64_t>(n, Jk[k]), Gt, 1, rows, Gnew, 1, rows, nullptr);
    if (k >= 2) {
      const double* Ak = (k == 2) ? s->G_of(fresh, 1) : s->A[k];
      double* Anext = (k == ks) ? nullptr : s->A[k + 1];
      plan_gemm(P, Pk[k - 1], I[k] * r[k], r[k - 1], Ak, 1, Pk[k - 1], Gnew, 1, r[k - 1], Anext, 1, Pk[k - 1],
                k == ks ? s->A32 : nullptr);
    } else if (ks == 1) {
      plan_copy(P, Gnew, nullptr, s->A32, Pk[1] * r[1]);
    }
  }

  P.steps.push_back({kStepPass2, 0, 0});

  // tail k = k*+1 .. m; the local solution has rank <= J_k
  int cur = 0;
  for (int k = ks + 1; k <= m; ++k) {
    const int64_t rows = r[k - 1] * I[k];
    const int64_t n = r[k];
    plan_gemm(P, rows, n, Jk[k], s->Y[cur], 1, rows, Bk(k), r[k], 1, s->Gt, 1, rows, nullptr);
    double* Gnew = s->G_of(fresh, k);
    plan_qr(P, s, rows, n, (int)std::min<int64_t>(n, Jk[k]), s->Gt, 1, rows, Gnew, 1, rows, nullptr);
    double* dst = (k == m) ? s->g_of(fresh) : s->Y[cur ^ 1];
    plan_gemm(P, n, Jk[k], rows, Gnew, rows, 1, s->Y[cur], 1, rows, dst, 1, n, nullptr);
    cur ^= 1;
  }
  if (ks == m) plan_copy(P, s->Y[0], s->g_of(fresh), nullptr, r[m]);

  {
    ttk::ChainOp op;
    op.type = ttk::kOpCommit;
    op.a = s->g_of(fresh);
    op.m = r[m];
    op.b = master;
    op.c = fresh;
    op.k = s->state_len;
    op.flag = s->flag;
    op.rejected = s->rejected;
    op.tdev = s->tdev;
    op.hist = s->hist;
    op.hist_cap = s->hist_cap;
    plan_chain(P, op);
  }
  // the update's result is committed here (an event marks it); then the next
  // update's steps 1-2 from the committed state (a rejected slice restored it)
  P.steps.push_back({kStepMark, 0, 0});
  plan_sweep(s, P, fresh);
}

// Steps 1-2 alone for the state in state[par]: run once before the first
// update and after tt_stream_set_state.
void build_sweep_plan(tt_stream* s, int par) {
  UpdatePlan& P = s->sweep0[par];
  P.ops.clear();
  P.wide_fma = wide_fma_of(s);
  P.steps.clear();
  plan_sweep(s, P, s->state[par]);
}

// Runs the steps of plan P of stream s with slice X.  trace (if not null)
// receives two stamps per chain operation; pass_ev (if not null) three events
// per pass: before it, after its contraction kernel, after its reduction.
tt_status run_steps(hipStream_t st, const tt_stream* s, const UpdatePlan& P, const void* X, tt_dtype xdt,
                    int64_t* trace, hipEvent_t const* pass_ev = nullptr, hipEvent_t mark_ev = nullptr) {
  const int ks = s->kstar;
  for (size_t si = 0; si < P.steps.size(); ++si) {
    const Step& step = P.steps[si];
    switch (step.kind) {
      case kStepChain:
        TT_HIP(ttk::chain_run(st, P.segs + si, 1, trace ? trace + 2 * step.first : nullptr));
        break;
      case kStepWide: {
        int64_t gx = 0;
        for (int q = step.first; q < step.first + step.count; ++q) {
          const ttk::ChainOp& o = P.ops[q];
          gx = std::max(gx, ttk::gemm64_blocks(o.m, o.n, o.k, o.ars, o.acs, o.brs, o.bcs, o.rho == ttk::kWideJb4));
        }
        TT_HIP(ttk::gemm64_ops(st, P.opptr + step.first, step.count, gx));
        break;
      }
      case kStepPass1: {
        if (pass_ev) TT_HIP(hipEventRecord(pass_ev[0], st));
        ttk::pass_mid_event() = pass_ev ? pass_ev[1] : nullptr;
        const hipError_t e =
            s->compute == TT_BF16
                ? ttk::pass1_bf16(st, X, xdt, s->p1b, s->Pk[ks], s->Jk[ks], (int)s->r[ks], s->B32, s->Z, s->ws,
                                  s->flag)
                : ttk::pass1(st, X, xdt, s->p1, s->Pk[ks], s->Jk[ks], (int)s->r[ks], s->B32, s->Z, s->ws, s->flag);
        ttk::pass_mid_event() = nullptr;
        TT_HIP(e);
        if (pass_ev) TT_HIP(hipEventRecord(pass_ev[2], st));
        break;
      }
      case kStepPass2: {
        if (pass_ev) TT_HIP(hipEventRecord(pass_ev[3], st));
        ttk::pass_mid_event() = pass_ev ? pass_ev[4] : nullptr;
        const hipError_t e =
            s->compute == TT_BF16
                ? ttk::pass2_bf16(st, X, xdt, s->p2b, s->Pk[ks], s->Jk[ks], (int)s->r[ks], s->A32, s->Y[0], s->ws2,
                                  s->flag)
                : ttk::pass2(st, X, xdt, s->Pk[ks], s->Jk[ks], (int)s->r[ks], s->A32, s->Y[0], s->flag);
        ttk::pass_mid_event() = nullptr;
        TT_HIP(e);
        if (pass_ev) TT_HIP(hipEventRecord(pass_ev[5], st));
        break;
      }
      case kStepMark:
        if (mark_ev) TT_HIP(hipEventRecord(mark_ev, st));
        break;
      default:
        return fail(TT_ERR_DEVICE, "corrupt update plan");
    }
  }
  return TT_OK;
}

tt_status run_plan(tt_stream* s, const void* X, tt_dtype xdt) {
  return run_steps(s->stream, s, s->plan[s->cur], X, xdt, s->trace, s->evpass[0] ? s->evpass : nullptr,
                   s->evcommit);
}

// Steps 1-2 of the first update from the committed state (after creation or
// set_state); stream-ordered.  Nothing to prepare for the ablation's plan.
tt_status run_first_sweep(tt_stream* s) {
  if (s->flags & TT_FLAG_NO_ORTHO) return TT_OK;
  return run_steps(s->stream, s, s->sweep0[s->cur], nullptr, TT_F32, nullptr);
}

}  // namespace

extern "C" {

const char* tt_last_error_string(void) { return g_last_error.c_str(); }

const char* tt_version(void) { return "tt_stream 0.1 (gfx950)"; }

tt_status tt_clamp_ranks(int32_t m, const int64_t* modes, const int64_t* ranks_in, int64_t* ranks_out) {
  if (!modes || !ranks_in || !ranks_out) return fail(TT_ERR_INVALID_ARG, "null pointer");
  tt_status st = check_shape(m, modes, ranks_in);
  if (st != TT_OK) return st;
  clamp(m, modes, ranks_in, ranks_out);
  return TT_OK;
}

tt_status tt_stream_create(const tt_stream_config* cfg, tt_stream** out) {
  if (!cfg || !out) return fail(TT_ERR_INVALID_ARG, "null cfg or out");
  *out = nullptr;
  if (!cfg->mode_sizes || !cfg->ranks) return fail(TT_ERR_INVALID_ARG, "null mode_sizes or ranks");
  const int m = cfg->n_slice_modes;
  tt_status st = check_shape(m, cfg->mode_sizes, cfg->ranks);
  if (st != TT_OK) return st;
  {
    std::vector<int64_t> cl(m);
    clamp(m, cfg->mode_sizes, cfg->ranks, cl.data());
    for (int k = 0; k < m; ++k)
      if (cl[k] != cfg->ranks[k])
        return fail(TT_ERR_RANK, "infeasible TT-ranks: need r_k <= r_{k-1} I_k and r_{k-1} <= I_k r_k");
  }
  if (cfg->compute != TT_F32 && cfg->compute != TT_BF16) return fail(TT_ERR_INVALID_ARG, "compute must be F32/BF16");
  if (cfg->flags & ~(TT_FLAG_SYNC_PUSH | TT_FLAG_PROFILE_OPS | TT_FLAG_AUTOTUNE | TT_FLAG_NO_ORTHO | TT_FLAG_WAVE_PLAN))
    return fail(TT_ERR_UNSUPPORTED, "unsupported flags");
  if (cfg->split_point < 0 || cfg->split_point > m) return fail(TT_ERR_INVALID_ARG, "split_point out of range");

  tt_stream* s = new (std::nothrow) tt_stream();
  if (!s) return fail(TT_ERR_OOM, "host allocation failed");
  s->m = m;
  s->compute = cfg->compute;
  s->flags = cfg->flags;
  s->stream = static_cast<hipStream_t>(cfg->hip_stream);
  if (cfg->allocator) {
    if (!cfg->allocator->alloc || !cfg->allocator->free) {
      delete s;
      return fail(TT_ERR_INVALID_ARG, "allocator needs alloc and free");
    }
    s->alloc = *cfg->allocator;
    s->has_alloc = true;
  }
  s->I.assign(m + 1, 1);
  s->r.assign(m + 1, 1);
  for (int k = 1; k <= m; ++k) {
    s->I[k] = cfg->mode_sizes[k - 1];
    s->r[k] = cfg->ranks[k - 1];
  }
  s->Pk.assign(m + 1, 1);
  s->Jk.assign(m + 1, 1);
  for (int k = 1; k <= m; ++k) s->Pk[k] = s->Pk[k - 1] * s->I[k];
  for (int k = m - 1; k >= 0; --k) s->Jk[k] = s->Jk[k + 1] * s->I[k + 1];
  s->N = s->Pk[m];
  s->coff.assign(m + 2, 0);
  for (int k = 1; k <= m; ++k) s->coff[k + 1] = s->coff[k] + s->r[k - 1] * s->I[k] * s->r[k];
  s->cores_len = s->coff[m + 1];
  s->state_len = s->cores_len + s->r[m];

  s->kstar = cfg->split_point > 0 ? cfg->split_point : choose_split(s);
  if (s->r[s->kstar] > 64) {
    delete s;
    return fail(TT_ERR_UNSUPPORTED, "rank at the split point must be <= 64");
  }
  if (s->flags & TT_FLAG_NO_ORTHO)
    for (int k = 1; k <= m; ++k)
      if (s->r[k] > 32 || (k < s->kstar && s->r[k] > s->Jk[k])) {
        delete s;
        return fail(TT_ERR_UNSUPPORTED,
                    "TT_FLAG_NO_ORTHO needs TT-ranks <= 32 and r_k <= I_{k+1}..I_m below the split point");
      }

  auto bail = [&](tt_status code, const std::string& msg) {
    release(s);
    delete s;
    return fail(code, msg);
  };
  if (hipGetDevice(&s->device) != hipSuccess) return bail(TT_ERR_DEVICE, "hipGetDevice failed");
  int lds = 65536;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device) != hipSuccess)
    return bail(TT_ERR_DEVICE, "cannot query LDS size");
  s->lds_limit = (size_t)lds;
  if (ttk::pass_setup() != hipSuccess || ttk::pass_bf16_setup() != hipSuccess ||
      ttk::chain_setup(s->lds_limit) != hipSuccess)
    return bail(TT_ERR_DEVICE, "kernel attribute setup failed");

  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
  if ((cfg->flags & TT_FLAG_AUTOTUNE) && cfg->split_point == 0 && !(s->flags & TT_FLAG_NO_ORTHO) &&
      !tune_split(s, cus))
    return bail(TT_ERR_DEVICE, "tuning the split point failed");

  const int m_ = m;
  const auto& I = s->I;
  const auto& r = s->r;
  const int ks = s->kstar;
  int64_t rmax = 1, qrmax = 1, gtmax = 1, ymax = 1;
  for (int k = 1; k <= m_; ++k) {
    rmax = std::max(rmax, r[k]);
    qrmax = std::max(qrmax, r[k - 1] * I[k] * r[k]);
    gtmax = std::max(gtmax, r[k - 1] * I[k] * r[k]);
  }
  for (int k = ks; k <= m_; ++k) ymax = std::max(ymax, r[k] * s->Jk[k]);

  {
    ttk::PassPlans plans = ttk::default_pass_plans(s->Pk[ks], s->Jk[ks], (int)r[ks], cus);
    if ((cfg->flags & TT_FLAG_AUTOTUNE) &&
        ttk::tuned_pass_plans(s->Pk[ks], s->Jk[ks], (int)r[ks], s->compute, cus, s->stream, &plans) != hipSuccess)
      return bail(TT_ERR_DEVICE, "tuning the slice passes failed");
    s->p1 = plans.p1;
    s->p1b = plans.p1b;
    s->p2b = plans.p2b;
  }
  const bool bf16 = s->compute == TT_BF16;

  // after the first failed allocation nothing more is requested
  bool ok = true;
  auto V = [&](size_t bytes) -> void* {
    void* p = ok ? dev_alloc(s, bytes) : nullptr;
    ok = ok && p;
    return p;
  };
  auto D = [&](size_t n) -> double* { return static_cast<double*>(V(n * sizeof(double))); };
  auto F = [&](size_t n) -> float* { return static_cast<float*>(V(n * sizeof(float))); };
  s->state[0] = D(s->state_len);
  s->state[1] = D(s->state_len);
  s->work = D(s->state_len);
  s->Rbuf = D(rmax * rmax);
  s->B.assign(m_ + 1, nullptr);
  for (int k = ks; k <= m_ - 1; ++k) s->B[k] = D(r[k] * s->Jk[k]);
  s->B32 = F(r[ks] * s->Jk[ks]);
  s->Z = D(s->Pk[ks] * r[ks]);
  s->Zk.assign(m_ + 1, nullptr);
  for (int k = 1; k < ks; ++k) s->Zk[k] = D(s->Pk[k] * r[k]);
  s->A.assign(m_ + 2, nullptr);
  for (int k = 3; k <= ks; ++k) s->A[k] = D(s->Pk[k - 1] * r[k - 1]);
  s->A32 = F(s->Pk[ks] * r[ks]);
  s->Gt = D(gtmax);
  s->Y[0] = D(ymax);
  s->Y[1] = D(ymax);
  s->qrwork = D(qrmax);
  if (s->flags & TT_FLAG_NO_ORTHO) {  // Gram matrices of the ablation
    s->GB.assign(m_ + 1, nullptr);
    s->GBi.assign(m_ + 1, nullptr);
    for (int k = 1; k <= m_; ++k) {
      s->GB[k] = D(r[k] * r[k]);
      s->GBi[k] = D(r[k] * r[k]);
    }
    s->gram_j = D(32 * 32);
    s->gram_ji = D(32 * 32);
    s->gram_tmp = D(std::max<int64_t>(qrmax, 2 * 32 * 32));
    s->gram_g = D(gtmax);
  }
  s->ws = bf16 ? static_cast<float*>(V(s->p1b.ws_bytes)) : F(s->p1.ws_floats);
  if (bf16) s->ws2 = static_cast<float*>(V(s->p2b.ws_bytes));
  s->flag = static_cast<int*>(V(sizeof(int) * 2));
  s->rejected = s->flag ? s->flag + 1 : nullptr;
  s->tdev = static_cast<int64_t*>(V(sizeof(int64_t)));
  if (cfg->keep_history) {
    s->hist_cap = cfg->history_capacity > 0 ? cfg->history_capacity : 1024;
    s->hist = D((size_t)s->hist_cap * r[m_]);
  }
  if (!ok || !s->flag || !s->tdev) return bail(TT_ERR_OOM, "device allocation failed");

#define TT_HIP_BAIL(call)                                                                   \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return bail(TT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
  TT_HIP_BAIL(hipMemsetAsync(s->flag, 0, sizeof(int) * 2, s->stream));
  TT_HIP_BAIL(hipMemsetAsync(s->tdev, 0, sizeof(int64_t), s->stream));
  TT_HIP_BAIL(hipEventCreate(&s->ev0));
  TT_HIP_BAIL(hipEventCreate(&s->ev1));
  TT_HIP_BAIL(hipEventCreateWithFlags(&s->evcopy, hipEventDisableTiming));
  TT_HIP_BAIL(hipEventCreate(&s->evcommit));

  std::vector<double> init(s->state_len);
  if (cfg->init_cores) std::memcpy(init.data(), cfg->init_cores, sizeof(double) * s->state_len);
  else normal_fill(init, cfg->seed);
  for (double v : init)
    if (!std::isfinite(v)) return bail(TT_ERR_NONFINITE, "initial cores contain NaN/Inf");
  TT_HIP_BAIL(hipMemcpyAsync(s->state[0], init.data(), sizeof(double) * s->state_len, hipMemcpyHostToDevice,
                             s->stream));
  s->cur = 0;
  for (int q = 0; q < 4; ++q) {
    const int par = q & 1;
    const bool sweep = q >= 2;
    if (sweep && (s->flags & TT_FLAG_NO_ORTHO)) continue;
    if (sweep) build_sweep_plan(s, par);
    else if (s->flags & TT_FLAG_NO_ORTHO) build_plan_noortho(s, par);
    else build_plan(s, par);
    UpdatePlan& P = sweep ? s->sweep0[par] : s->plan[par];
    for (const ttk::ChainOp& op : P.ops)
      if (!ttk::chain_op_supported(op)) return bail(TT_ERR_UNSUPPORTED, "a core re-orthogonalisation exceeds 256 columns");
    // one device block: ops, then a segment per step, then a pointer per op
    const size_t nops = P.ops.size(), nsteps = P.steps.size();
    const size_t b_ops = sizeof(ttk::ChainOp) * nops, b_segs = sizeof(ttk::ChainSeg) * nsteps;
    char* blk = static_cast<char*>(dev_alloc(s, b_ops + b_segs + sizeof(ttk::ChainOp*) * nops));
    if (!blk) return bail(TT_ERR_OOM, "plan allocation failed");
    P.dev = reinterpret_cast<ttk::ChainOp*>(blk);
    P.segs = reinterpret_cast<ttk::ChainSeg*>(blk + b_ops);
    P.opptr = reinterpret_cast<ttk::ChainOp**>(blk + b_ops + b_segs);
    std::vector<char> host(b_ops + b_segs + sizeof(ttk::ChainOp*) * nops);
    std::memcpy(host.data(), P.ops.data(), b_ops);
    for (size_t i = 0; i < nsteps; ++i) {
      ttk::ChainSeg sg{P.dev + P.steps[i].first, P.steps[i].kind == kStepChain ? P.steps[i].count : 0, 0};
      std::memcpy(host.data() + b_ops + i * sizeof(sg), &sg, sizeof(sg));
    }
    for (size_t i = 0; i < nops; ++i) {
      ttk::ChainOp* q = P.dev + i;
      std::memcpy(host.data() + b_ops + b_segs + i * sizeof(q), &q, sizeof(q));
    }
    TT_HIP_BAIL(hipMemcpy(blk, host.data(), host.size(), hipMemcpyHostToDevice));
  }
  if (s->flags & TT_FLAG_PROFILE_OPS) {
    s->trace_len = (int64_t)std::max(s->plan[0].ops.size(), s->plan[1].ops.size());
    s->trace = static_cast<int64_t*>(dev_alloc(s, sizeof(int64_t) * 2 * s->trace_len));
    if (!s->trace) return bail(TT_ERR_OOM, "profile buffer");
    TT_HIP_BAIL(hipMemsetAsync(s->trace, 0, sizeof(int64_t) * 2 * s->trace_len, s->stream));
    (void)hipDeviceGetAttribute(&s->wall_khz, hipDeviceAttributeWallClockRate, s->device);
    if (s->wall_khz <= 0) s->wall_khz = 100000;
    for (hipEvent_t& e : s->evpass) TT_HIP_BAIL(hipEventCreate(&e));
  }
  {
    const tt_status st0 = run_first_sweep(s);
    if (st0 != TT_OK) return bail(st0, g_last_error);
  }
  TT_HIP_BAIL(hipStreamSynchronize(s->stream));
#undef TT_HIP_BAIL
  ttk::handle_register(s, ttk::kHandleStream);
  *out = s;
  return TT_OK;
}

tt_status tt_stream_push_slice(tt_stream* s, const void* slice, tt_dtype dtype, int on_device) {
  if (!valid(s)) return fail(TT_ERR_INVALID_ARG, "invalid handle");
  if (!slice) return fail(TT_ERR_INVALID_ARG, "null slice");
  if (dtype != TT_F64 && dtype != TT_F32 && dtype != TT_BF16) return fail(TT_ERR_INVALID_ARG, "bad dtype");
  if (s->server) return fail(TT_ERR_STATE, "the stream is registered with a server; submit its slices there");
  const void* X = slice;
  if (!on_device) {
    const size_t bytes = (size_t)s->N * dtype_size(dtype);
    if (s->stage_bytes < bytes) {
      void* p = dev_alloc(s, bytes);
      if (!p) return fail(TT_ERR_OOM, "staging allocation failed");
      s->stage = p;
      s->stage_bytes = bytes;
    }
    TT_HIP(hipMemcpyAsync(s->stage, slice, bytes, hipMemcpyHostToDevice, s->stream));
    TT_HIP(hipEventRecord(s->evcopy, s->stream));
    X = s->stage;
  }
  TT_HIP(hipEventRecord(s->ev0, s->stream));
  tt_status st = run_plan(s, X, dtype);
  if (st != TT_OK) return st;
  s->traced_plan = s->cur;
  s->cur ^= 1;
  TT_HIP(hipEventRecord(s->ev1, s->stream));
  s->timed = true;
  s->pushes++;
  if (!on_device) TT_HIP(hipEventSynchronize(s->evcopy));
  if (s->flags & TT_FLAG_SYNC_PUSH) return tt_stream_synchronize(s);
  return TT_OK;
}

tt_status tt_stream_wait_update(tt_stream* s) {
  if (!valid(s)) return fail(TT_ERR_INVALID_ARG, "invalid handle");
  if (s->server) {  // a lane runs its updates
    TT_HIP(ttk::stream_quiesce(s));
    return TT_OK;
  }
  if (s->pushes == 0) return TT_OK;
  TT_HIP(hipEventSynchronize((s->flags & TT_FLAG_NO_ORTHO) ? s->ev1 : s->evcommit));
  return TT_OK;
}

tt_status tt_stream_synchronize(tt_stream* s) {
  if (!valid(s)) return fail(TT_ERR_INVALID_ARG, "invalid handle");
  TT_HIP(ttk::stream_quiesce(s));
  int rej = 0;
  TT_HIP(hipMemcpy(&rej, s->rejected, sizeof(int), hipMemcpyDeviceToHost));
  if (rej > s->rejected_seen) {
    s->rejected_seen = rej;
    return fail(TT_ERR_NONFINITE, "a slice contained NaN/Inf; its update was discarded");
  }
  return TT_OK;
}

tt_status tt_stream_time(tt_stream* s, int64_t* t_out) {
  if (!valid(s) || !t_out) return fail(TT_ERR_INVALID_ARG, "invalid handle or null output");
  TT_HIP(ttk::stream_quiesce(s));
  TT_HIP(hipMemcpy(t_out, s->tdev, sizeof(int64_t), hipMemcpyDeviceToHost));
  return TT_OK;
}

tt_status tt_stream_info(const tt_stream* s, int64_t* cores_len, int64_t* r_last, int32_t* split_point,
                         int64_t* device_bytes) {
  if (!valid(s)) return fail(TT_ERR_INVALID_ARG, "invalid handle");
  if (cores_len) *cores_len = s->cores_len;
  if (r_last) *r_last = s->r[s->m];
  if (split_point) *split_point = s->kstar;
  if (device_bytes) *device_bytes = (int64_t)s->device_bytes;
  return TT_OK;
}

tt_status tt_stream_get_state(tt_stream* s, double* cores, double* g, int64_t* t_out) {
  if (!valid(s)) return fail(TT_ERR_INVALID_ARG, "invalid handle");
  TT_HIP(ttk::stream_quiesce(s));
  if (cores) TT_HIP(hipMemcpy(cores, s->master(), sizeof(double) * s->cores_len, hipMemcpyDeviceToHost));
  if (g) TT_HIP(hipMemcpy(g, s->g_of(s->master()), sizeof(double) * s->r[s->m], hipMemcpyDeviceToHost));
  if (t_out) TT_HIP(hipMemcpy(t_out, s->tdev, sizeof(int64_t), hipMemcpyDeviceToHost));
  return TT_OK;
}

tt_status tt_stream_set_state(tt_stream* s, const double* cores, const double* g, int64_t t) {
  if (!valid(s) || !cores || !g) return fail(TT_ERR_INVALID_ARG, "invalid handle or null input");
  if (t < 0) return fail(TT_ERR_INVALID_ARG, "t must be >= 0");
  for (int64_t i = 0; i < s->cores_len; ++i)
    if (!std::isfinite(cores[i])) return fail(TT_ERR_NONFINITE, "cores contain NaN/Inf");
  for (int64_t i = 0; i < s->r[s->m]; ++i)
    if (!std::isfinite(g[i])) return fail(TT_ERR_NONFINITE, "g contains NaN/Inf");
  TT_HIP(ttk::stream_quiesce(s));
  TT_HIP(hipMemcpy(s->master(), cores, sizeof(double) * s->cores_len, hipMemcpyHostToDevice));
  TT_HIP(hipMemcpy(s->g_of(s->master()), g, sizeof(double) * s->r[s->m], hipMemcpyHostToDevice));
  TT_HIP(hipMemcpy(s->tdev, &t, sizeof(int64_t), hipMemcpyHostToDevice));
  s->hist_t0 = t;  // the ring holds no row of the new state's past
  // the next update's steps 1-2 were prepared from the replaced state
  const tt_status st = run_first_sweep(s);
  if (st != TT_OK) return st;
  TT_HIP(hipStreamSynchronize(s->stream));
  return TT_OK;
}

tt_status tt_stream_get_history(tt_stream* s, double* out, int64_t rows, int64_t* rows_out) {
  if (!valid(s) || !out || !rows_out) return fail(TT_ERR_INVALID_ARG, "invalid handle or null output");
  if (!s->hist) return fail(TT_ERR_STATE, "history was not enabled");
  int64_t t = 0;
  TT_HIP(ttk::stream_quiesce(s));
  TT_HIP(hipMemcpy(&t, s->tdev, sizeof(int64_t), hipMemcpyDeviceToHost));
  // rows written since creation or the last set_state: update u wrote row u % hist_cap
  const int64_t have = std::min(std::max<int64_t>(t - s->hist_t0, 0), s->hist_cap);
  const int64_t n = std::min(have, rows);
  const int64_t rm = s->r[s->m];
  std::vector<double> ring((size_t)s->hist_cap * rm);
  TT_HIP(hipMemcpy(ring.data(), s->hist, sizeof(double) * ring.size(), hipMemcpyDeviceToHost));
  const int64_t first = t - have;  // oldest kept update index
  for (int64_t i = 0; i < n; ++i) {
    const int64_t row = (first + i) % s->hist_cap;
    std::memcpy(out + i * rm, ring.data() + row * rm, sizeof(double) * rm);
  }
  *rows_out = n;
  return TT_OK;
}

tt_status tt_stream_reconstruct(tt_stream* s, void* out, tt_dtype dtype, int on_device) {
  if (!valid(s) || !out) return fail(TT_ERR_INVALID_ARG, "invalid handle or null output");
  if (dtype != TT_F64 && dtype != TT_F32) return fail(TT_ERR_INVALID_ARG, "reconstruct dtype must be F64/F32");
  int64_t t = 0;
  TT_HIP(ttk::stream_quiesce(s));
  TT_HIP(hipMemcpy(&t, s->tdev, sizeof(int64_t), hipMemcpyDeviceToHost));
  if (t == 0) return fail(TT_ERR_STATE, "no slice has been pushed");
  if (!s->recon[0] || !s->recon[1]) {
    if (!s->recon[0]) s->recon[0] = static_cast<double*>(dev_alloc(s, sizeof(double) * s->N));
    if (s->recon[0] && !s->recon[1]) s->recon[1] = static_cast<double*>(dev_alloc(s, sizeof(double) * s->N));
    if (!s->recon[0] || !s->recon[1]) return fail(TT_ERR_OOM, "reconstruction buffers");
  }
  hipStream_t st = s->stream;
  // V_{m+1} = g; V_k = G_k^L V_{k+1}, viewed as r_{k-1} x (I_k .. I_m)
  const double* V = s->g_of(s->master());
  int64_t cols = 1;
  int cur = 0;
  for (int k = s->m; k >= 1; --k) {
    const int64_t rows = s->r[k - 1] * s->I[k];
    double* dst = s->recon[cur];
    TT_HIP(ttk::gemm64(st, rows, cols, s->r[k], s->G_of(s->master(), k), 1, rows, V, 1, s->r[k], dst, 1, rows,
                       nullptr));
    V = dst;
    cols *= s->I[k];
    cur ^= 1;
  }
  if (on_device) {
    TT_HIP(ttk::convert_out(st, V, out, dtype, s->N));
  } else {
    if (dtype == TT_F64) {
      TT_HIP(hipMemcpyAsync(out, V, sizeof(double) * s->N, hipMemcpyDeviceToHost, st));
    } else {
      double* tmp = s->recon[cur];
      TT_HIP(ttk::convert_out(st, V, tmp, TT_F32, s->N));
      TT_HIP(hipMemcpyAsync(out, tmp, sizeof(float) * s->N, hipMemcpyDeviceToHost, st));
    }
    TT_HIP(hipStreamSynchronize(st));
  }
  return TT_OK;
}

tt_status tt_stream_last_push_ms(tt_stream* s, float* ms) {
  if (!valid(s) || !ms) return fail(TT_ERR_INVALID_ARG, "invalid handle or null output");
  if (!s->timed) return fail(TT_ERR_STATE, "no push yet");
  hipEvent_t end = (s->flags & TT_FLAG_NO_ORTHO) ? s->ev1 : s->evcommit;
  TT_HIP(hipEventSynchronize(end));
  TT_HIP(hipEventElapsedTime(ms, s->ev0, end));
  return TT_OK;
}

tt_status tt_stream_op_profile(tt_stream* s, int64_t cap, int32_t* kinds, int64_t* dims, double* us,
                               int64_t* count) {
  if (!valid(s) || !count || (cap > 0 && (!kinds || !dims || !us))) return fail(TT_ERR_INVALID_ARG, "null argument");
  if (!s->trace) return fail(TT_ERR_STATE, "stream was not created with TT_FLAG_PROFILE_OPS");
  if (s->traced_plan < 0) return fail(TT_ERR_STATE, "no push yet");
  TT_HIP(ttk::stream_quiesce(s));
  const UpdatePlan& P = s->plan[s->traced_plan];
  std::vector<int64_t> stamps(2 * P.ops.size());
  TT_HIP(hipMemcpy(stamps.data(), s->trace, sizeof(int64_t) * stamps.size(), hipMemcpyDeviceToHost));
  // ops launched over the whole GPU are not timed here
  std::vector<int> chain_ops;
  for (const Step& step : P.steps)
    if (step.kind == kStepChain)
      for (int i = step.first; i < step.first + step.count; ++i) chain_ops.push_back(i);
  *count = (int64_t)chain_ops.size();
  const int64_t n = std::min<int64_t>(cap, *count);
  for (int64_t q = 0; q < n; ++q) {
    const int i = chain_ops[q];
    const ttk::ChainOp& o = P.ops[i];
    kinds[q] = o.type;
    dims[3 * q] = o.m;
    dims[3 * q + 1] = o.n;
    dims[3 * q + 2] = o.type == ttk::kOpQr ? o.rho : o.k;
    us[q] = (double)(stamps[2 * i + 1] - stamps[2 * i]) * 1000.0 / (double)s->wall_khz;
  }
  return TT_OK;
}

tt_status tt_stream_pass_profile(tt_stream* s, float* ms) {
  if (!valid(s) || !ms) return fail(TT_ERR_INVALID_ARG, "null argument");
  if (!s->evpass[0]) return fail(TT_ERR_STATE, "stream was not created with TT_FLAG_PROFILE_OPS");
  if (s->traced_plan < 0) return fail(TT_ERR_STATE, "no push yet");
  TT_HIP(hipEventSynchronize(s->evpass[5]));
  TT_HIP(hipEventElapsedTime(ms + 0, s->evpass[0], s->evpass[1]));
  TT_HIP(hipEventElapsedTime(ms + 1, s->evpass[0], s->evpass[2]));
  TT_HIP(hipEventElapsedTime(ms + 2, s->evpass[3], s->evpass[4]));
  TT_HIP(hipEventElapsedTime(ms + 3, s->evpass[3], s->evpass[5]));
  return TT_OK;
}

tt_status tt_stream_pass_kernels(const tt_stream* s, int32_t* pass1, int32_t* pass2) {
  if (!valid(s) || !pass1 || !pass2) return fail(TT_ERR_INVALID_ARG, "null argument");
  const bool bf16 = s->compute == TT_BF16;
  *pass1 = bf16 ? 1 : 0;
  const int ks = s->kstar;
  *pass2 = bf16 ? (s->p2b.staged ? 2 : 1) : (ttk::pass2_grouped(s->Pk[ks], s->Jk[ks], (int)s->r[ks], TT_F32) ? 3 : 0);
  return TT_OK;
}

tt_status tt_stream_time_passes(tt_stream* s, const void* const* slices, int32_t nslices, tt_dtype dtype,
                                int32_t reps, float* us) {
  if (!valid(s) || !slices || !us) return fail(TT_ERR_INVALID_ARG, "null argument");
  if (nslices < 1) return fail(TT_ERR_INVALID_ARG, "no slices");
  for (int32_t i = 0; i < nslices; ++i)
    if (!slices[i]) return fail(TT_ERR_INVALID_ARG, "null slice");
  if (dtype != TT_F64 && dtype != TT_F32 && dtype != TT_BF16) return fail(TT_ERR_INVALID_ARG, "bad dtype");
  if (reps < 1 || reps > 100000) return fail(TT_ERR_INVALID_ARG, "reps out of range");
  if (s->pushes == 0) return fail(TT_ERR_STATE, "no push yet");
  if (s->server) return fail(TT_ERR_STATE, "the stream is registered with a server");
  const int ks = s->kstar;
  const int64_t P = s->Pk[ks], J = s->Jk[ks];
  const int r = (int)s->r[ks];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  tt_status st = TT_OK;
  auto pass = [&](int which, int i) -> hipError_t {
    const void* slice = slices[i % nslices];
    if (which == 1)
      return s->compute == TT_BF16
                 ? ttk::pass1_bf16(s->stream, slice, dtype, s->p1b, P, J, r, s->B32, s->Z, s->ws, s->flag)
                 : ttk::pass1(s->stream, slice, dtype, s->p1, P, J, r, s->B32, s->Z, s->ws, s->flag);
    return s->compute == TT_BF16
               ? ttk::pass2_bf16(s->stream, slice, dtype, s->p2b, P, J, r, s->A32, s->Y[0], s->ws2, s->flag)
               : ttk::pass2(s->stream, slice, dtype, P, J, r, s->A32, s->Y[0], s->flag);
  };
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int q = 0; q < 4 && e == hipSuccess; ++q) {
    ttk::pass_launch_mask() = 1 + (q & 1);  // contraction kernel, then reduction
    e = pass(1 + q / 2, 0);                 // warm launch
    if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = pass(1 + q / 2, i + 1);
    if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    us[q] = ms * 1000.f / (float)reps;
  }
  ttk::pass_launch_mask() = 3;
  // the passes' outputs are per-update scratch; the flag is zero between
  // updates (the commit clears it) and may have been set by a timed launch
  if (e == hipSuccess) e = hipMemsetAsync(s->flag, 0, sizeof(int), s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) st = fail(TT_ERR_DEVICE, hipGetErrorString(e));
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}

tt_status tt_stream_destroy(tt_stream* s) {
  if (!valid(s)) return fail(TT_ERR_INVALID_ARG, "invalid handle");
  (void)ttk::stream_quiesce(s);
  if (s->server) ttk::server_forget(s->server, s->server_id);
  ttk::handle_unregister(s);
  release(s);
  s->magic = kDead;
  delete s;
  return TT_OK;
}

}  // extern "C"
