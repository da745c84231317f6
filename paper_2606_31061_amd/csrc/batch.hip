// Batches (include/tt_batch.h) and the serving loop (include/tt_server.h).
//
// A wave is one update of each of its member streams with launches shared by
// all members, whatever their shapes: every member's update steps are cut at
// the two slice passes into three phases; inside a phase a member alternates
// chain segments and whole-GPU products, and slot w of every member's phase
// runs in one launch (chain segment w on one workgroup per member, then
// product w of the members that have one).  A member with fewer products than
// the longest may start its phase a few slots late (align_members), so that
// the members' long chain segments share launches.  Each pass runs as one launch per
// kernel template shape over the members of that shape.  Per wave, the
// members' operation-list pointers, slices and pass sizes go to the device in
// one descriptor upload.  Every member computes exactly what it computes
// alone: the same operations, kernels, launch shapes and arithmetic order.
//
// A batch is a fixed wave pushed again and again (optionally replayed from
// HIP graphs).  A server builds a new wave for each launch from the requests
// it admits and keeps up to `lanes` waves in flight on its own HIP streams.
#include "stream_internal.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <vector>

using ttk::fail_msg;

constexpr uint64_t kDeadMagic = 0xdeadbeefdeadbeefULL;

namespace ttk {
namespace {

enum WaveLaunchKind { kWlChain = 0, kWlWide = 1, kWlPass1 = 2, kWlPass2 = 3 };
struct WaveLaunch {
  int kind = 0;
  int phase = 0, slot = 0;       // chain/wide: phase and slot
  std::vector<int> members;      // participating members (wave order)
  size_t off = 0;                // descriptor offset in the upload
  int64_t gx = 0;                // wide: grid.x; passes: main grid.x
  unsigned grx = 0;              // passes: reduction grid.x
  int rep = -1;                  // passes: a member whose plan gives the template shape
};
// Per member and phase: chain segments (first, count) and, between them,
// whole-GPU product op indices (segments = products + 1).
struct MemberPhase {
  std::vector<std::pair<int, int>> segs;
  std::vector<int> wides;
};

// A stream of the batch's own beside its HIP stream, and the events that fork
// a run of launches onto it and join them back.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

struct Wave {
  std::vector<tt_stream*> members;
  std::vector<std::array<MemberPhase, 3>> phases;
  std::vector<WaveLaunch> launches;
  size_t bytes = 0;  // descriptor upload
};

// Template shape of a member's pass launch (members of one launch share it).
std::array<int, 5> pass_key(const tt_stream* s, int pass) {
  const int ks = s->kstar;
  const int ntn = s->r[ks] <= 32 ? 1 : 2;
  if (s->compute == TT_BF16) {
    if (pass == 1) return {1, 1, s->p1b.vec, s->p1b.waves, ntn};
    return {1, 2, pass2b_vx(s->Pk[ks]) ? 1 : 0, s->p2b.staged ? -1 : s->p2b.waves, ntn};
  }
  if (pass == 1) return {0, 1, s->p1.vec, s->p1.waves, s->p1.ntn};
  return {0, 2, pass2_vec(s->Pk[ks]), pass2_grouped(s->Pk[ks], s->Jk[ks], (int)s->r[ks], TT_F32) ? pass2g_nwt(s->Pk[ks]) : 0,
          ntn};
}

void pass_grids(const tt_stream* s, int pass, int64_t* gx, unsigned* grx) {
  const int ks = s->kstar;
  unsigned a = 0, b = 0;
  if (s->compute == TT_BF16) {
    if (pass == 1) pass1b_grids(s->p1b, &a, &b);
    else pass2b_grids(s->p2b, &a, &b);
  } else if (pass == 1) {
    pass1_grids(s->p1, s->Pk[ks], &a, &b);
  } else {
    a = pass2_grid(s->Jk[ks]);
  }
  *gx = a;
  *grx = b;
}

PassDesc pass_desc(const tt_stream* s, int pass, const void* x) {
  const int ks = s->kstar;
  PassDesc d{};
  d.x = x;
  d.w = pass == 1 ? s->B32 : s->A32;
  d.out = pass == 1 ? s->Z : s->Y[0];
  d.ws = pass == 1 ? s->ws : s->ws2;
  d.flag = s->flag;
  d.P = s->Pk[ks];
  d.J = s->Jk[ks];
  d.r = (int32_t)s->r[ks];
  if (s->compute == TT_BF16) {
    const PassBPlan& pl = pass == 1 ? s->p1b : s->p2b;
    d.tiles = pl.tiles;
    d.chunks = pl.chunks;
  } else {
    d.tiles = (int32_t)((d.P + 32 * s->p1.vec - 1) / (32 * s->p1.vec));
    d.chunks = s->p1.chunks;
  }
  return d;
}

// A rough device time (us) of one chain operation on its workgroup, from its
// shape: only the ordering of the heavy operations (tall QRs) matters to the
// alignment below.
double op_cost_us(const ChainOp& o) {
  const double m = (double)o.m, n = (double)o.n, k = (double)o.k;
  switch (o.type) {
    case kOpQr: {
      if (o.rho == 1) return 3.0 + 0.012 * m;
      if (m <= 512) return 15.0 + 0.032 * m;
      const bool capped = o.rho >= 2 && o.rho < o.n && !o.r;  // plus a one-pass completion
      return (capped ? 1.15 : 1.0) * (10.0 + 0.042 * m * (n > 16 ? 1.0 : 0.75));
    }
    case kOpGemm: {
      double c = m * n * k / 3e4;
      if (m * n <= 1024) c = std::max(c, 0.035 * k);
      c = std::max(c, 0.0065 * m);
      return 1.5 + c;
    }
    case kOpNormG: return 2.0 + 0.00027 * k;
    case kOpCopy: return 1.0 + 0.0001 * m;
    case kOpCommit: return 1.0 + 0.0001 * k;
    default: return 5.0;
  }
}

// Members of a wave whose phase has fewer whole-GPU products than the
// longest start it later (empty chain segments first), by an offset chosen
// so that the members' heavy chain segments share launches: each launch
// lasts as long as its slowest segment, so the sum over launches of the
// slowest estimated segment is reduced by coordinate descent from the
// left-aligned start.  The members' own operations and their order are
// unchanged.
void align_members(Wave& w) {
  const int n = (int)w.members.size();
  for (int ph = 0; ph < 3; ++ph) {
    size_t W = 0;
    for (int i = 0; i < n; ++i) W = std::max(W, w.phases[i][ph].wides.size());
    if (W == 0) continue;
    const int S = (int)W + 1;
    std::vector<std::vector<double>> c(n);
    std::vector<int> range(n), d(n, 0);
    for (int i = 0; i < n; ++i) {
      const auto& mp = w.phases[i][ph];
      const auto& ops = w.members[i]->plan[0].ops;
      for (const auto& sg : mp.segs) {
        double t = 0.0;
        for (int q = sg.first; q < sg.first + sg.second; ++q) t += op_cost_us(ops[q]);
        c[i].push_back(t);
      }
      range[i] = (int)(W - mp.wides.size());
    }
    auto total = [&]() {
      double sum = 0.0;
      for (int sl = 0; sl < S; ++sl) {
        double mx = 0.0;
        for (int i = 0; i < n; ++i) {
          const int j = sl - d[i];
          if (j >= 0 && j < (int)c[i].size()) mx = std::max(mx, c[i][j]);
        }
        sum += mx;
      }
      return sum;
    };
    double best = total();
    for (int pass = 0; pass < 4; ++pass) {
      bool moved = false;
      for (int i = 0; i < n; ++i) {
        if (range[i] == 0) continue;
        const int d0 = d[i];
        int bd = d0;
        for (int dd = 0; dd <= range[i]; ++dd) {
          if (dd == d0) continue;
          d[i] = dd;
          const double t = total();
          if (t < best - 1e-9) {
            best = t;
            bd = dd;
          }
        }
        d[i] = bd;
        moved = moved || bd != d0;
      }
      if (!moved) break;
    }
    for (int i = 0; i < n; ++i) {
      if (d[i] == 0) continue;
      auto& mp = w.phases[i][ph];
      mp.segs.insert(mp.segs.begin(), d[i], std::pair<int, int>{0, 0});
      mp.wides.insert(mp.wides.begin(), d[i], -1);
    }
  }
}

// The launch sequence of a wave (its shape depends only on the members).
void wave_build(Wave& w) {
  const int n = (int)w.members.size();
  w.phases.assign(n, {});
  for (int i = 0; i < n; ++i) {
    const UpdatePlan& P = w.members[i]->plan[0];
    int ph = 0;
    auto& mp = w.phases[i];
    for (auto& x : mp) x.segs.push_back({0, 0});
    for (const Step& st : P.steps) {
      if (st.kind == kStepChain) {
        auto& sg = mp[ph].segs.back();
        if (sg.second > 0 && sg.first + sg.second == st.first) sg.second += st.count;  // split only by a mark
        else sg = {st.first, st.count};
      } else if (st.kind == kStepWide) {
        for (int q = 0; q < st.count; ++q) {  // a joined launch of the stream: one slot per product
          mp[ph].wides.push_back(st.first + q);
          mp[ph].segs.push_back({0, 0});
        }
      } else if (st.kind == kStepMark) {
        // the commit mark: no work, and no boundary for a wave
      } else {
        ++ph;
      }
    }
  }
  align_members(w);
  w.launches.clear();
  size_t off = 0;
  auto add = [&](WaveLaunch&& L, size_t bytes) {
    L.off = off;
    off += (bytes + 255) & ~size_t(255);
    w.launches.push_back(std::move(L));
  };
  for (int ph = 0; ph < 3; ++ph) {
    size_t W = 0;
    for (int i = 0; i < n; ++i) W = std::max(W, w.phases[i][ph].wides.size());
    for (size_t sl = 0; sl <= W; ++sl) {
      bool any = false;
      for (int i = 0; i < n; ++i) {
        const auto& mp = w.phases[i][ph];
        any = any || (sl < mp.segs.size() && mp.segs[sl].second > 0);
      }
      if (any) {
        WaveLaunch L;
        L.kind = kWlChain;
        L.phase = ph;
        L.slot = (int)sl;
        for (int i = 0; i < n; ++i) L.members.push_back(i);
        add(std::move(L), sizeof(ChainSeg) * n);
      }
      if (sl < W) {
        WaveLaunch L;
        L.kind = kWlWide;
        L.phase = ph;
        L.slot = (int)sl;
        for (int i = 0; i < n; ++i) {
          const auto& mp = w.phases[i][ph];
          if (sl < mp.wides.size() && mp.wides[sl] >= 0) {
            L.members.push_back(i);
            const ChainOp& o = w.members[i]->plan[0].ops[mp.wides[sl]];
            L.gx = std::max(L.gx, gemm64_blocks(o.m, o.n, o.k, o.ars, o.acs, o.brs, o.bcs, o.rho == kWideJb4));
          }
        }
        const size_t k = L.members.size();
        add(std::move(L), sizeof(ChainOp*) * k);
      }
    }
    if (ph < 2) {
      const int pass = ph + 1;
      std::vector<std::array<int, 5>> keys;
      std::vector<std::vector<int>> groups;
      for (int i = 0; i < n; ++i) {
        const auto key = pass_key(w.members[i], pass);
        size_t g = 0;
        while (g < keys.size() && keys[g] != key) ++g;
        if (g == keys.size()) {
          keys.push_back(key);
          groups.emplace_back();
        }
        groups[g].push_back(i);
      }
      for (auto& grp : groups) {
        WaveLaunch L;
        L.kind = pass == 1 ? kWlPass1 : kWlPass2;
        L.members = grp;
        L.rep = grp[0];
        for (int i : grp) {
          int64_t gx;
          unsigned grx;
          pass_grids(w.members[i], pass, &gx, &grx);
          L.gx = std::max(L.gx, gx);
          L.grx = std::max(L.grx, grx);
        }
        const size_t k = L.members.size();
        add(std::move(L), sizeof(PassDesc) * k);
      }
    }
  }
  w.bytes = off;
}

// The wave's descriptors for the members' current parities and slices.
void wave_fill(const Wave& w, char* h, const void* const* slices) {
  const int n = (int)w.members.size();
  for (const WaveLaunch& L : w.launches) {
    char* p = h + L.off;
    if (L.kind == kWlChain) {
      ChainSeg* sg = reinterpret_cast<ChainSeg*>(p);
      for (int i = 0; i < n; ++i) {
        const tt_stream* s = w.members[i];
        const auto& mp = w.phases[i][L.phase];
        const auto seg = L.slot < (int)mp.segs.size() ? mp.segs[L.slot] : std::pair<int, int>{0, 0};
        sg[i] = ChainSeg{s->plan[s->cur].dev + seg.first, seg.second, 0};
      }
    } else if (L.kind == kWlWide) {
      ChainOp** op = reinterpret_cast<ChainOp**>(p);
      for (size_t k = 0; k < L.members.size(); ++k) {
        const int i = L.members[k];
        const tt_stream* s = w.members[i];
        op[k] = s->plan[s->cur].dev + w.phases[i][L.phase].wides[L.slot];
      }
    } else {
      const int pass = L.kind == kWlPass1 ? 1 : 2;
      PassDesc* pd = reinterpret_cast<PassDesc*>(p);
      for (size_t k = 0; k < L.members.size(); ++k)
        pd[k] = pass_desc(w.members[L.members[k]], pass, slices[L.members[k]]);
    }
  }
}

// Enqueues the descriptor upload from host buffer h and every launch.  With
// a side stream, a run of slice-pass launches (one per pass plan, different
// members, so independent) forks when it holds launches of fewer than
// kNarrowBlocks blocks, which leave most of the GPU idle: those go to the side
// stream and run beside the wider ones, and the run joins before the next
// chain launch.  Under graph capture the fork and join become edges of the
// graph.  Which stream a launch takes changes no result.
constexpr int64_t kNarrowBlocks = 256;
tt_status wave_enqueue(const Wave& w, hipStream_t st, char* dev, const char* h, tt_dtype dtype, const SideStream* side) {
  const int n = (int)w.members.size();
  TT_HIP_RT(hipMemcpyAsync(dev, h, w.bytes, hipMemcpyHostToDevice, st));
  const auto is_pass = [](const WaveLaunch& L) { return L.kind == kWlPass1 || L.kind == kWlPass2; };
  const auto narrow = [](const WaveLaunch& L) { return L.gx * (int64_t)L.members.size() < kNarrowBlocks; };
  const size_t nl = w.launches.size();
  hipStream_t run_side = nullptr;  // the side stream while a forked run lasts
  size_t run_end = 0;
  for (size_t li = 0; li < nl; ++li) {
    const WaveLaunch& L = w.launches[li];
    if (side && is_pass(L) && li >= run_end) {
      size_t e = li;
      int nn = 0;
      while (e < nl && w.launches[e].kind == L.kind) nn += narrow(w.launches[e++]) ? 1 : 0;
      run_end = e;
      if (nn > 0 && e - li >= 2) {
        TT_HIP_RT(hipEventRecord(side->fork, st));
        TT_HIP_RT(hipStreamWaitEvent(side->stream, side->fork, 0));
        run_side = side->stream;
      }
    }
    hipStream_t ls = (run_side && narrow(L)) ? run_side : st;
    char* p = dev + L.off;
    const int k = (int)L.members.size();
    if (L.kind == kWlChain) {
      TT_HIP_RT(chain_run(ls, reinterpret_cast<const ChainSeg*>(p), n));
    } else if (L.kind == kWlWide) {
      TT_HIP_RT(gemm64_ops(ls, reinterpret_cast<const ChainOp* const*>(p), k, L.gx));
    } else {
      const tt_stream* s = w.members[L.rep];
      const int ks = s->kstar;
      PassLaunch bl{reinterpret_cast<const PassDesc*>(p), k, (unsigned)L.gx, L.grx};
      const int64_t P = s->Pk[ks], J = s->Jk[ks];
      const int r = (int)s->r[ks];
      if (L.kind == kWlPass1) {
        if (s->compute == TT_BF16)
          TT_HIP_RT(pass1_bf16(ls, nullptr, dtype, s->p1b, P, J, r, nullptr, nullptr, nullptr, nullptr, &bl));
        else
          TT_HIP_RT(pass1(ls, nullptr, dtype, s->p1, P, J, r, nullptr, nullptr, nullptr, nullptr, &bl));
      } else {
        if (s->compute == TT_BF16)
          TT_HIP_RT(pass2_bf16(ls, nullptr, dtype, s->p2b, P, J, r, nullptr, nullptr, nullptr, nullptr, &bl));
        else
          TT_HIP_RT(pass2(ls, nullptr, dtype, P, J, r, nullptr, nullptr, nullptr, &bl));
      }
    }
    if (run_side && li + 1 == run_end) {  // join the run
      TT_HIP_RT(hipEventRecord(side->join, run_side));
      TT_HIP_RT(hipStreamWaitEvent(st, side->join, 0));
      run_side = nullptr;
    }
  }
  return TT_OK;
}

// The members' committed state moves to the other buffer (host bookkeeping,
// after their updates are enqueued).
void wave_commit(Wave& w) {
  for (tt_stream* s : w.members) {
    s->cur ^= 1;
    s->pushes++;
  }
}

// Same update structure: shapes, split point, precision, pass plans and ops.
bool same_structure(const tt_stream* a, const tt_stream* b) {
  if (a->m != b->m || a->kstar != b->kstar || a->I != b->I || a->r != b->r || a->compute != b->compute) return false;
  const auto same1 = [](const Pass1Plan& x, const Pass1Plan& y) {
    return x.vec == y.vec && x.ntn == y.ntn && x.waves == y.waves && x.chunks == y.chunks;
  };
  const auto sameb = [](const PassBPlan& x, const PassBPlan& y) {
    return x.vec == y.vec && x.ntn == y.ntn && x.waves == y.waves && x.chunks == y.chunks;
  };
  if (!same1(a->p1, b->p1) || !sameb(a->p1b, b->p1b) || !sameb(a->p2b, b->p2b)) return false;
  const UpdatePlan &pa = a->plan[0], &pb = b->plan[0];
  if (pa.ops.size() != pb.ops.size() || pa.steps.size() != pb.steps.size()) return false;
  for (size_t i = 0; i < pa.steps.size(); ++i)
    if (pa.steps[i].kind != pb.steps[i].kind || pa.steps[i].first != pb.steps[i].first ||
        pa.steps[i].count != pb.steps[i].count)
      return false;
  for (size_t i = 0; i < pa.ops.size(); ++i) {
    const ChainOp &x = pa.ops[i], &y = pb.ops[i];
    if (x.type != y.type || x.m != y.m || x.n != y.n || x.k != y.k || x.rho != y.rho) return false;
  }
  return true;
}

}  // namespace
}  // namespace ttk

// ====================================================================== batch

constexpr uint64_t kBatchMagic = 0x54544241544348ULL;  // "TTBATCH"
constexpr int kBatchSlots = 8;

struct tt_batch {
  uint64_t magic = kBatchMagic;
  hipStream_t stream = nullptr;
  ttk::SideStream side;  // narrow slice-pass launches run here, beside the rest
  ttk::Wave wave;
  int n_groups = 0;  // distinct update structures (informational)
  char* dev = nullptr;
  char* host[kBatchSlots] = {};
  hipEvent_t done[kBatchSlots] = {};
  bool used[kBatchSlots] = {};
  hipGraphExec_t graph[kBatchSlots] = {};  // per slot, when graph replay is on
  tt_dtype graph_dtype[kBatchSlots] = {};   // slice type the slot's graph was captured for
  bool use_graph = false;
  int next = 0;
  std::vector<int> rejected_seen;
};

namespace {

bool batch_valid(const tt_batch* b) {
  return b != nullptr && ttk::handle_live(b, ttk::kHandleBatch) && b->magic == kBatchMagic;
}

void batch_drop_graphs(tt_batch* b) {
  for (hipGraphExec_t& g : b->graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

void batch_release(tt_batch* b) {
  batch_drop_graphs(b);
  if (b->side.stream) (void)hipStreamDestroy(b->side.stream);
  if (b->side.fork) (void)hipEventDestroy(b->side.fork);
  if (b->side.join) (void)hipEventDestroy(b->side.join);
  b->side = ttk::SideStream{};
  if (b->dev) (void)hipFree(b->dev);
  b->dev = nullptr;
  for (int k = 0; k < kBatchSlots; ++k) {
    if (b->done[k]) (void)hipEventDestroy(b->done[k]);
    if (b->host[k]) (void)hipHostFree(b->host[k]);
    b->done[k] = nullptr;
    b->host[k] = nullptr;
  }
}

}  // namespace

extern "C" {

tt_status tt_batch_create(tt_stream* const* streams, int32_t n, void* hip_stream, tt_batch** out) {
  if (!streams || !out || n < 1) return fail_msg(TT_ERR_INVALID_ARG, "null argument or n < 1");
  if (n > 65535) return fail_msg(TT_ERR_INVALID_ARG, "at most 65535 streams per batch");
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail_msg(TT_ERR_DEVICE, "hipGetDevice failed");
  for (int i = 0; i < n; ++i) {
    const tt_stream* s = streams[i];
    if (!ttk::stream_valid(s)) return fail_msg(TT_ERR_INVALID_ARG, "invalid stream handle");
    if (s->device != dev) return fail_msg(TT_ERR_INVALID_ARG, "stream lives on another device");
    if (s->stream != static_cast<hipStream_t>(hip_stream))
      return fail_msg(TT_ERR_INVALID_ARG, "stream uses another HIP stream");
    if (s->trace) return fail_msg(TT_ERR_INVALID_ARG, "streams with TT_FLAG_PROFILE_OPS cannot be batched");
    if (s->server) return fail_msg(TT_ERR_STATE, "stream is registered with a server");
    for (int j = 0; j < i; ++j)
      if (streams[j] == s) return fail_msg(TT_ERR_INVALID_ARG, "duplicate stream");
  }
  tt_batch* b = new (std::nothrow) tt_batch();
  if (!b) return fail_msg(TT_ERR_OOM, "host allocation failed");
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->wave.members.assign(streams, streams + n);
  b->rejected_seen.resize(n);
  std::vector<int> reps;
  for (int i = 0; i < n; ++i) {
    bool seen = false;
    for (int j : reps) seen = seen || ttk::same_structure(streams[j], streams[i]);
    if (!seen) reps.push_back(i);
    b->rejected_seen[i] = streams[i]->rejected_seen;
  }
  b->n_groups = (int)reps.size();
  ttk::wave_build(b->wave);
  void* d = nullptr;
  if (hipMalloc(&d, b->wave.bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete b;
    return fail_msg(TT_ERR_OOM, "batch descriptor allocation failed");
  }
  b->dev = static_cast<char*>(d);
  if (hipStreamCreateWithFlags(&b->side.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->side.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->side.join, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    batch_release(b);
    delete b;
    return fail_msg(TT_ERR_DEVICE, "batch side stream creation failed");
  }
  for (int q = 0; q < kBatchSlots; ++q) {
    void* h = nullptr;
    if (hipHostMalloc(&h, b->wave.bytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->done[q], hipEventDisableTiming) != hipSuccess) {
      if (h) (void)hipHostFree(h);
      batch_release(b);
      delete b;
      return fail_msg(TT_ERR_OOM, "batch staging allocation failed");
    }
    b->host[q] = static_cast<char*>(h);
  }
  ttk::handle_register(b, ttk::kHandleBatch);
  *out = b;
  return TT_OK;
}

tt_status tt_batch_push(tt_batch* b, const void* const* slices, tt_dtype dtype) {
  if (!batch_valid(b) || !slices) return fail_msg(TT_ERR_INVALID_ARG, "invalid batch or null slices");
  if (dtype != TT_F64 && dtype != TT_F32 && dtype != TT_BF16) return fail_msg(TT_ERR_INVALID_ARG, "bad dtype");
  const int n = (int)b->wave.members.size();
  for (int i = 0; i < n; ++i)
    if (!slices[i]) return fail_msg(TT_ERR_INVALID_ARG, "null slice");
  // descriptors of this push into a free pinned slot, then one upload
  const int q = b->next;
  b->next = (b->next + 1) % kBatchSlots;
  if (b->used[q]) TT_HIP_RT(hipEventSynchronize(b->done[q]));
  char* h = b->host[q];
  ttk::wave_fill(b->wave, h, slices);
  if (b->use_graph && b->graph[q] && b->graph_dtype[q] != dtype) {  // kernels depend on the slice type
    (void)hipGraphExecDestroy(b->graph[q]);
    b->graph[q] = nullptr;
  }
  if (b->use_graph && !b->graph[q]) {
    hipGraph_t g = nullptr;
    TT_HIP_RT(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const tt_status st = ttk::wave_enqueue(b->wave, b->stream, b->dev, h, dtype, &b->side);
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st != TT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    TT_HIP_RT(e);
    const hipError_t ei = hipGraphInstantiate(&b->graph[q], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    TT_HIP_RT(ei);
    b->graph_dtype[q] = dtype;
  }
  if (b->use_graph) {
    TT_HIP_RT(hipGraphLaunch(b->graph[q], b->stream));
  } else {
    const tt_status st = ttk::wave_enqueue(b->wave, b->stream, b->dev, h, dtype, &b->side);
    if (st != TT_OK) return st;
  }
  TT_HIP_RT(hipEventRecord(b->done[q], b->stream));
  b->used[q] = true;
  ttk::wave_commit(b->wave);
  return TT_OK;
}

tt_status tt_batch_synchronize(tt_batch* b, int32_t* rejected) {
  if (!batch_valid(b)) return fail_msg(TT_ERR_INVALID_ARG, "invalid batch");
  TT_HIP_RT(hipStreamSynchronize(b->stream));
  bool any = false;
  for (size_t i = 0; i < b->wave.members.size(); ++i) {
    tt_stream* s = b->wave.members[i];
    int rej = 0;
    TT_HIP_RT(hipMemcpy(&rej, s->rejected, sizeof(int), hipMemcpyDeviceToHost));
    const int fresh = rej - b->rejected_seen[i];
    if (rejected) rejected[i] = fresh;
    if (fresh > 0) any = true;
    b->rejected_seen[i] = rej;
    s->rejected_seen = rej;
  }
  return any ? fail_msg(TT_ERR_NONFINITE, "a slice contained NaN/Inf; its stream's update was discarded") : TT_OK;
}

tt_status tt_batch_use_graph(tt_batch* b, int32_t enable) {
  if (!batch_valid(b)) return fail_msg(TT_ERR_INVALID_ARG, "invalid batch");
  if (enable && b->stream == nullptr)
    return fail_msg(TT_ERR_UNSUPPORTED, "graph replay needs a batch on a non-default HIP stream");
  TT_HIP_RT(hipStreamSynchronize(b->stream));
  if (!enable) batch_drop_graphs(b);
  b->use_graph = enable != 0;
  return TT_OK;
}

tt_status tt_batch_info(const tt_batch* b, int32_t* n_streams, int32_t* n_groups) {
  if (!batch_valid(b)) return fail_msg(TT_ERR_INVALID_ARG, "invalid batch");
  if (n_streams) *n_streams = (int32_t)b->wave.members.size();
  if (n_groups) *n_groups = (int32_t)b->n_groups;
  return TT_OK;
}

tt_status tt_batch_destroy(tt_batch* b) {
  if (!batch_valid(b)) return fail_msg(TT_ERR_INVALID_ARG, "invalid batch");
  (void)hipStreamSynchronize(b->stream);
  ttk::handle_unregister(b);
  batch_release(b);
  b->magic = kDeadMagic;
  delete b;
  return TT_OK;
}

}  // extern "C"

// ===================================================================== server


constexpr uint64_t kServerMagic = 0x5454534552564552ULL;  // "TTSERVER"
constexpr int kMaxLanes = 8;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int id;
  const void* slice;
  tt_dtype dtype;
  uint64_t tag;
  uint64_t bytes;
  Clock::time_point t0;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* dev = nullptr;        // descriptor upload
  char* host = nullptr;       // pinned
  size_t cap = 0;
  int* rej_host = nullptr;    // pinned: members' rejected counters after the wave
  size_t rej_cap = 0;
  bool busy = false;
  ttk::Wave wave;
  std::vector<Request> reqs;  // wave order
};

struct Result {
  uint64_t tag;
  double latency;
  int rejected;
};

}  // namespace

struct tt_server {
  uint64_t magic = kServerMagic;
  int max_wave = 1;
  uint64_t budget = 0;
  std::vector<Lane> lanes;
  std::vector<tt_stream*> streams;
  std::vector<int> in_flight;       // per stream: requests in flight (0 or 1)
  std::vector<int> queued;          // per stream: requests queued
  std::vector<int> rejected_seen;   // per stream
  std::deque<Request> queue;
  std::deque<Result> results;
  uint64_t bytes_admitted = 0, peak_bytes = 0;
  int64_t waves = 0, retired = 0, n_in_flight = 0;
};

namespace {

bool server_valid(const tt_server* s) {
  return s != nullptr && ttk::handle_live(s, ttk::kHandleServer) && s->magic == kServerMagic;
}

void lane_release(Lane& L) {
  if (L.stream) (void)hipStreamSynchronize(L.stream);
  if (L.done) (void)hipEventDestroy(L.done);
  if (L.dev) (void)hipFree(L.dev);
  if (L.host) (void)hipHostFree(L.host);
  if (L.rej_host) (void)hipHostFree(L.rej_host);
  if (L.stream) (void)hipStreamDestroy(L.stream);
  L = Lane{};
}

// Retires the lane's wave if it has finished (or waits for it).
tt_status lane_retire(tt_server* sv, Lane& L, bool wait, int* done) {
  if (!L.busy) return TT_OK;
  if (wait) {
    TT_HIP_RT(hipEventSynchronize(L.done));
  } else {
    const hipError_t q = hipEventQuery(L.done);
    if (q == hipErrorNotReady) return TT_OK;
    TT_HIP_RT(q);
  }
  const auto now = Clock::now();
  for (size_t k = 0; k < L.reqs.size(); ++k) {
    const Request& r = L.reqs[k];
    const int rej = L.rej_host[k] - sv->rejected_seen[r.id];
    sv->rejected_seen[r.id] = L.rej_host[k];
    if (sv->streams[r.id]) sv->streams[r.id]->rejected_seen = L.rej_host[k];
    sv->results.push_back(Result{r.tag, std::chrono::duration<double>(now - r.t0).count(), rej > 0 ? 1 : 0});
    sv->in_flight[r.id] = 0;
    sv->bytes_admitted -= r.bytes;
  }
  sv->retired += (int64_t)L.reqs.size();
  sv->n_in_flight -= (int64_t)L.reqs.size();
  if (done) *done += (int)L.reqs.size();
  L.reqs.clear();
  L.wave.members.clear();
  L.busy = false;
  return TT_OK;
}

// Admits queued requests into a wave and launches it on lane L.
tt_status lane_launch(tt_server* sv, Lane& L) {
  std::vector<Request> pick;
  std::vector<char> blocked(sv->streams.size(), 0);  // an earlier request of the stream is still queued
  tt_dtype dt = TT_F32;
  for (auto it = sv->queue.begin(); it != sv->queue.end() && (int)pick.size() < sv->max_wave;) {
    const Request& r = *it;
    bool ok = !blocked[r.id] && !sv->in_flight[r.id];
    if (ok && !pick.empty() && r.dtype != dt) ok = false;
    if (ok && sv->budget && sv->bytes_admitted + r.bytes > sv->budget &&
        !(sv->bytes_admitted == 0 && pick.empty()))
      ok = false;
    if (!ok) {
      blocked[r.id] = 1;
      ++it;
      continue;
    }
    if (pick.empty()) dt = r.dtype;
    pick.push_back(r);
    sv->in_flight[r.id] = 1;
    sv->queued[r.id] -= 1;
    sv->bytes_admitted += r.bytes;
    blocked[r.id] = 1;
    it = sv->queue.erase(it);
  }
  if (pick.empty()) return TT_OK;
  sv->peak_bytes = std::max(sv->peak_bytes, sv->bytes_admitted);
  L.wave.members.clear();
  std::vector<const void*> slices;
  for (const Request& r : pick) {
    L.wave.members.push_back(sv->streams[r.id]);
    slices.push_back(r.slice);
  }
  ttk::wave_build(L.wave);
  if (L.wave.bytes > L.cap) {  // grow the lane's descriptor buffers (the lane is idle)
    if (L.dev) (void)hipFree(L.dev);
    if (L.host) (void)hipHostFree(L.host);
    L.dev = nullptr;
    L.host = nullptr;
    L.cap = 0;
    const size_t cap = std::max(L.wave.bytes, size_t(1) << 16);
    void* d = nullptr;
    void* h = nullptr;
    if (hipMalloc(&d, cap) != hipSuccess) {
      (void)hipGetLastError();
      return fail_msg(TT_ERR_OOM, "server descriptor buffer");
    }
    if (hipHostMalloc(&h, cap, hipHostMallocDefault) != hipSuccess) {
      (void)hipFree(d);
      return fail_msg(TT_ERR_OOM, "server staging buffer");
    }
    L.dev = static_cast<char*>(d);
    L.host = static_cast<char*>(h);
    L.cap = cap;
  }
  if (pick.size() > L.rej_cap) {
    if (L.rej_host) (void)hipHostFree(L.rej_host);
    L.rej_host = nullptr;
    void* h = nullptr;
    const size_t cap = std::max<size_t>(pick.size(), 64);
    if (hipHostMalloc(&h, cap * sizeof(int), hipHostMallocDefault) != hipSuccess)
      return fail_msg(TT_ERR_OOM, "server staging buffer");
    L.rej_host = static_cast<int*>(h);
    L.rej_cap = cap;
  }
  ttk::wave_fill(L.wave, L.host, slices.data());
  tt_status st = ttk::wave_enqueue(L.wave, L.stream, L.dev, L.host, dt, nullptr);
  if (st != TT_OK) return st;
  for (size_t k = 0; k < pick.size(); ++k)
    TT_HIP_RT(hipMemcpyAsync(L.rej_host + k, L.wave.members[k]->rejected, sizeof(int), hipMemcpyDeviceToHost,
                             L.stream));
  TT_HIP_RT(hipEventRecord(L.done, L.stream));
  // calls on a member's handle (state, reconstruction, destroy) wait for this wave
  for (tt_stream* m : L.wave.members) m->ext_done = L.done;
  ttk::wave_commit(L.wave);
  L.reqs = std::move(pick);
  L.busy = true;
  sv->waves += 1;
  sv->n_in_flight += (int64_t)L.reqs.size();
  return TT_OK;
}

uint64_t slice_bytes(const tt_stream* s, tt_dtype dt) {
  const uint64_t e = dt == TT_F64 ? 8 : (dt == TT_F32 ? 4 : 2);
  return (uint64_t)s->N * e;
}

}  // namespace

extern "C" {

tt_status tt_server_create(const tt_server_config* cfg, tt_server** out) {
  if (!cfg || !out) return fail_msg(TT_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (cfg->max_wave < 1 || cfg->max_wave > 65535) return fail_msg(TT_ERR_INVALID_ARG, "max_wave out of range");
  if (cfg->lanes < 1 || cfg->lanes > kMaxLanes) return fail_msg(TT_ERR_INVALID_ARG, "lanes out of range");
  tt_server* sv = new (std::nothrow) tt_server();
  if (!sv) return fail_msg(TT_ERR_OOM, "host allocation failed");
  sv->max_wave = cfg->max_wave;
  sv->budget = cfg->hbm_budget;
  sv->lanes.resize(cfg->lanes);
  for (Lane& L : sv->lanes) {
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
      for (Lane& M : sv->lanes) lane_release(M);
      delete sv;
      return fail_msg(TT_ERR_DEVICE, "server lane creation failed");
    }
  }
  ttk::handle_register(sv, ttk::kHandleServer);
  *out = sv;
  return TT_OK;
}

tt_status tt_server_add(tt_server* sv, tt_stream* s, int32_t* id) {
  if (!server_valid(sv) || !ttk::stream_valid(s) || !id) return fail_msg(TT_ERR_INVALID_ARG, "invalid argument");
  if (s->trace) return fail_msg(TT_ERR_INVALID_ARG, "streams with TT_FLAG_PROFILE_OPS cannot be served");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s->device)
    return fail_msg(TT_ERR_INVALID_ARG, "stream lives on another device");
  for (const tt_stream* t : sv->streams)
    if (t == s) return fail_msg(TT_ERR_INVALID_ARG, "stream already registered");
  if (s->server) return fail_msg(TT_ERR_STATE, "stream is registered with another server");
  // the stream's own earlier work completes before the server's lanes use it
  TT_HIP_RT(hipStreamSynchronize(s->stream));
  *id = (int32_t)sv->streams.size();
  s->server = sv;
  s->server_id = *id;
  sv->streams.push_back(s);
  sv->in_flight.push_back(0);
  sv->queued.push_back(0);
  sv->rejected_seen.push_back(s->rejected_seen);
  return TT_OK;
}

tt_status tt_server_submit(tt_server* sv, int32_t id, const void* slice, tt_dtype dtype, uint64_t tag) {
  if (!server_valid(sv) || !slice) return fail_msg(TT_ERR_INVALID_ARG, "invalid argument");
  if (id < 0 || id >= (int32_t)sv->streams.size()) return fail_msg(TT_ERR_INVALID_ARG, "unknown stream id");
  if (!sv->streams[id]) return fail_msg(TT_ERR_INVALID_ARG, "the stream of this id was destroyed");
  if (dtype != TT_F64 && dtype != TT_F32 && dtype != TT_BF16) return fail_msg(TT_ERR_INVALID_ARG, "bad dtype");
  sv->queue.push_back(Request{id, slice, dtype, tag, slice_bytes(sv->streams[id], dtype), Clock::now()});
  sv->queued[id] += 1;
  return TT_OK;
}

tt_status tt_server_poll(tt_server* sv, int32_t* done) {
  if (!server_valid(sv)) return fail_msg(TT_ERR_INVALID_ARG, "invalid server");
  int d = 0;
  for (Lane& L : sv->lanes) {
    const tt_status st = lane_retire(sv, L, false, &d);
    if (st != TT_OK) return st;
  }
  for (Lane& L : sv->lanes) {
    if (sv->queue.empty()) break;
    if (L.busy) continue;
    const tt_status st = lane_launch(sv, L);
    if (st != TT_OK) return st;
  }
  if (done) *done = d;
  return TT_OK;
}

tt_status tt_server_drain(tt_server* sv) {
  if (!server_valid(sv)) return fail_msg(TT_ERR_INVALID_ARG, "invalid server");
  for (;;) {
    const tt_status st = tt_server_poll(sv, nullptr);
    if (st != TT_OK) return st;
    bool busy = false;
    for (const Lane& L : sv->lanes) busy = busy || L.busy;
    if (!busy && sv->queue.empty()) return TT_OK;
    if (busy) {  // wait for the oldest busy lane rather than spinning
      for (Lane& L : sv->lanes)
        if (L.busy) {
          const tt_status st2 = lane_retire(sv, L, true, nullptr);
          if (st2 != TT_OK) return st2;
          break;
        }
    }
  }
}

tt_status tt_server_take(tt_server* sv, int64_t cap, uint64_t* tags, double* latency_s, int32_t* rejected,
                         int64_t* n) {
  if (!server_valid(sv) || !n || (cap > 0 && (!tags || !latency_s || !rejected)))
    return fail_msg(TT_ERR_INVALID_ARG, "invalid argument");
  int64_t k = 0;
  while (k < cap && !sv->results.empty()) {
    const Result& r = sv->results.front();
    tags[k] = r.tag;
    latency_s[k] = r.latency;
    rejected[k] = r.rejected;
    sv->results.pop_front();
    ++k;
  }
  *n = k;
  return TT_OK;
}

tt_status tt_server_stats(const tt_server* sv, int64_t* waves, int64_t* retired, int64_t* queued,
                          int64_t* in_flight, uint64_t* peak_bytes) {
  if (!server_valid(sv)) return fail_msg(TT_ERR_INVALID_ARG, "invalid server");
  if (waves) *waves = sv->waves;
  if (retired) *retired = sv->retired;
  if (queued) *queued = (int64_t)sv->queue.size();
  if (in_flight) *in_flight = sv->n_in_flight;
  if (peak_bytes) *peak_bytes = sv->peak_bytes;
  return TT_OK;
}

tt_status tt_server_destroy(tt_server* sv) {
  if (!server_valid(sv)) return fail_msg(TT_ERR_INVALID_ARG, "invalid server");
  for (Lane& L : sv->lanes) lane_release(L);
  for (tt_stream* s : sv->streams)
    if (s) {  // the lanes (and their events) are gone; the stream is its own again
      s->server = nullptr;
      s->server_id = -1;
      s->ext_done = nullptr;
    }
  ttk::handle_unregister(sv);
  sv->magic = kDeadMagic;
  delete sv;
  return TT_OK;
}

}  // extern "C"

void ttk::server_forget(tt_server* sv, int32_t id) {
  if (!server_valid(sv) || id < 0 || id >= (int32_t)sv->streams.size()) return;
  for (auto it = sv->queue.begin(); it != sv->queue.end();) {
    if (it->id == id) {
      it = sv->queue.erase(it);
      sv->queued[id] -= 1;
    } else {
      ++it;
    }
  }
  sv->streams[id] = nullptr;
}
