// Tile-shape tuner of the two slice passes.
//
// The passes' tunable launch shapes (rows per lane, waves per block, and how
// many blocks split the reduction) are picked per stream shape (P, J, r) and
// contraction precision by timing candidate shapes on the device once per
// process; the result is cached, so every stream of that shape, alone or in
// a batch, runs the same plan and computes the same bits.  The choice
// depends only on the shape.  The cached record also keeps the time of the
// two passes with the chosen shapes, which the runtime compares across split
// points.
#include "tt_internal.h"

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace ttk {
namespace {

using Key = std::tuple<int64_t, int64_t, int, int>;
std::mutex g_mu;
std::map<Key, PassPlans> g_cache;

// Chunk counts whose tiles x chunks blocks fill the chip about half, once,
// twice and four times: for each, the largest count that stays within that
// many blocks (no CU gets one block more than the others) and the smallest
// that reaches it.
std::vector<int> fill_counts(int tiles, int cus, int64_t max_chunks) {
  std::vector<int> out;
  for (int f : {1, 2, 4, 8}) {
    const int64_t target = (int64_t)cus * f / 2;
    for (int64_t c : {target / tiles, (target + tiles - 1) / tiles}) {
      if (c > max_chunks) c = max_chunks;
      if (c < 1) c = 1;
      bool seen = false;
      for (int v : out) seen = seen || v == (int)c;
      if (!seen) out.push_back((int)c);
    }
  }
  return out;
}

template <class Launch>
float time_plan(hipStream_t st, hipEvent_t e0, hipEvent_t e1, Launch launch) {
  for (int i = 0; i < 2; ++i)
    if (launch() != hipSuccess) return -1.f;
  if (hipEventRecord(e0, st) != hipSuccess) return -1.f;
  constexpr int kReps = 8;
  for (int i = 0; i < kReps; ++i)
    if (launch() != hipSuccess) return -1.f;
  if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.f;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.f;
  return ms / kReps;
}

struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  void* get(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    ptrs.push_back(p);
    return p;
  }
};

// Times the candidates of one stream shape; false if the device work failed.
bool tune(int64_t P, int64_t J, int r, tt_dtype compute, int cus, hipStream_t st, PassPlans& best) {
  const bool bf16 = compute == TT_BF16;
  const int ntn = r <= 32 ? 1 : 2;
  std::vector<Pass1Plan> c1;
  std::vector<PassBPlan> c1b, c2b;
  if (!bf16) {
    const int64_t pairs = (J + 1) / 2;
    const std::vector<std::pair<int, int>> shapes =
        ntn == 1 ? std::vector<std::pair<int, int>>{{4, 8}, {4, 4}, {2, 8}, {2, 4}, {1, 16}, {1, 8}}
                 : std::vector<std::pair<int, int>>{{2, 4}, {1, 8}};
    for (auto [vec, waves] : shapes) {
      if (P % vec != 0) continue;
      Pass1Plan pl;
      pl.vec = vec;
      pl.ntn = ntn;
      pl.waves = waves;
      pl = finish_plan(pl, P);
      for (int c : fill_counts(pl.tiles, cus, std::max<int64_t>(1, pairs / (4 * waves)))) {
        pl.chunks = c;
        c1.push_back(finish_plan(pl, P));
      }
    }
  } else {
    for (int vec : {8, 4, 2, 1}) {
      if (vec != 1 && P % vec != 0) continue;
      if (vec == 8 && ntn != 1) continue;
      PassBPlan pl;
      pl.vec = vec;
      pl.ntn = ntn;
      pl.waves = 4;
      pl = pass1b_finish(pl, P, J);
      for (int c : fill_counts(pl.tiles, cus, std::max<int64_t>(1, (J + 15) / 16 / 4))) {
        pl.chunks = c;
        c1b.push_back(pass1b_finish(pl, P, J));
      }
    }
    if (P % 8 == 0) {  // the staged pass 2
      PassBPlan pl;
      pl.ntn = ntn;
      pl.staged = 1;
      c2b.push_back(pass2b_finish(pl, P, J));
    }
    for (int waves : {4, 8}) {
      if (waves == 8 && ntn != 1) continue;
      PassBPlan pl;
      pl.ntn = ntn;
      pl.waves = waves;
      pl = pass2b_finish(pl, P, J);
      const int64_t nsb = (P + 63) / 64;
      for (int c : {1, 2, 3, 4, 6}) {
        if (c > nsb) continue;
        pl.chunks = c;
        c2b.push_back(pass2b_finish(pl, P, J));
      }
    }
  }
  size_t ws = 256;
  for (const auto& p : c1) ws = std::max(ws, p.ws_floats * sizeof(float));
  for (const auto& p : c1b) ws = std::max(ws, p.ws_bytes);
  for (const auto& p : c2b) ws = std::max(ws, p.ws_bytes);
  Scratch sc;
  const size_t xbytes = (size_t)P * J * (bf16 ? 2 : 4);
  void* X = sc.get(xbytes);
  float* W1 = static_cast<float*>(sc.get((size_t)r * J * 4));
  float* W2 = static_cast<float*>(sc.get((size_t)P * r * 4));
  double* Z = static_cast<double*>(sc.get((size_t)P * r * 8));
  double* Y = static_cast<double*>(sc.get((size_t)r * J * 8));
  void* W = sc.get(ws);
  int* flag = static_cast<int*>(sc.get(4));
  if (!X || !W1 || !W2 || !Z || !Y || !W || !flag) return false;
  // finite operands: ones
  if (bf16) {
    if (hipMemsetD16Async((hipDeviceptr_t)X, 0x3F80, (size_t)P * J, st) != hipSuccess) return false;
  } else if (hipMemsetD32Async((hipDeviceptr_t)X, 0x3F800000, (size_t)P * J, st) != hipSuccess) {
    return false;
  }
  if (hipMemsetD32Async((hipDeviceptr_t)W1, 0x3F800000, (size_t)r * J, st) != hipSuccess ||
      hipMemsetD32Async((hipDeviceptr_t)W2, 0x3F800000, (size_t)P * r, st) != hipSuccess ||
      hipMemsetAsync(flag, 0, 4, st) != hipSuccess)
    return false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return false;
  bool ok = true;
  float bt = 1e30f, total = 0.f;
  for (const auto& p : c1) {
    const float ms = time_plan(st, e0, e1, [&] {
      return pass1(st, X, TT_F32, p, P, J, r, W1, Z, static_cast<float*>(W), flag);
    });
    if (ms < 0) ok = false;
    if (ms >= 0 && ms < bt) {
      bt = ms;
      best.p1 = p;
    }
  }
  if (!bf16) {
    const float ms = time_plan(st, e0, e1, [&] { return pass2(st, X, TT_F32, P, J, r, W2, Y, flag); });
    if (ms < 0) ok = false;
    total = bt + ms;
  }
  bt = 1e30f;
  for (const auto& p : c1b) {
    const float ms = time_plan(st, e0, e1, [&] { return pass1_bf16(st, X, TT_BF16, p, P, J, r, W1, Z, W, flag); });
    if (ms < 0) ok = false;
    if (ms >= 0 && ms < bt) {
      bt = ms;
      best.p1b = p;
    }
  }
  if (bf16) total = bt;
  bt = 1e30f;
  for (const auto& p : c2b) {
    const float ms = time_plan(st, e0, e1, [&] { return pass2_bf16(st, X, TT_BF16, p, P, J, r, W2, Y, W, flag); });
    if (ms < 0) ok = false;
    if (ms >= 0 && ms < bt) {
      bt = ms;
      best.p2b = p;
    }
  }
  if (bf16) total += bt;
  best.ms = total;
  (void)hipStreamSynchronize(st);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ok;
}

}  // namespace

PassPlans default_pass_plans(int64_t P, int64_t J, int r, int cus) {
  PassPlans p;
  p.p1 = pass1_plan(P, J, r, cus);
  p.p1b = pass1b_plan(P, J, r, cus);
  p.p2b = pass2b_plan(P, J, r, cus);
  return p;
}

hipError_t tuned_pass_plans(int64_t P, int64_t J, int r, tt_dtype compute, int cus, hipStream_t st,
                            PassPlans* out) {
  const Key key{P, J, r, (int)compute};
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_cache.find(key);
  if (it != g_cache.end()) {
    *out = it->second;
    return hipSuccess;
  }
  PassPlans p = default_pass_plans(P, J, r, cus);
  if (!tune(P, J, r, compute, cus, st, p)) return hipErrorLaunchFailure;
  p.tuned = true;
  g_cache[key] = p;
  *out = p;
  return hipSuccess;
}

}  // namespace ttk
