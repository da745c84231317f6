// Host-side definitions shared by the stream runtime (tt_stream.hip) and the
// batch and serving runtime (batch.hip): one stream's handle and its planned
// update.
#pragma once

#include "tt_internal.h"
#include "tt_batch.h"
#include "tt_server.h"

#include <string>
#include <vector>

namespace ttk {

constexpr uint64_t kStreamMagic = 0x54545354524d3031ULL;  // "TTSTRM01"

// The update as a sequence of steps over its operation list: chain segments
// (operations first .. first + count - 1 on one workgroup), whole-GPU
// products (operation first) and the two slice passes.
// kStepMark: no work; the single-stream path records the commit event there
// (the update's result is final; later steps prepare the next update).
enum StepKind { kStepChain = 0, kStepWide = 1, kStepPass1 = 2, kStepPass2 = 3, kStepMark = 4 };
struct Step {
  int kind;
  int first;
  int count;
};
struct UpdatePlan {
  std::vector<ttk::ChainOp> ops;
  std::vector<Step> steps;
  double wide_fma = 2.0e5;         // products from this size run as whole-GPU launches
  ttk::ChainOp* dev = nullptr;     // the ops on the device
  ttk::ChainSeg* segs = nullptr;   // segs[i]: step i's operations (device; chain steps)
  ttk::ChainOp** opptr = nullptr;  // opptr[i] = dev + i (device)
};


}  // namespace ttk

struct tt_stream {
  uint64_t magic = ttk::kStreamMagic;
  int m = 0;
  std::vector<int64_t> I;    // I[1..m] (I[0] unused)
  std::vector<int64_t> r;    // r[0..m], r[0] = 1
  std::vector<int64_t> Pk;   // Pk[k] = I_1..I_k, Pk[0] = 1
  std::vector<int64_t> Jk;   // Jk[k] = I_{k+1}..I_m, Jk[m] = 1
  std::vector<int64_t> coff; // offset of G_k in a state buffer; coff[m+1] = offset of g
  int64_t N = 0, cores_len = 0, state_len = 0;
  int kstar = 1;
  tt_dtype compute = TT_F32;
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  tt_allocator alloc{};
  bool has_alloc = false;
  size_t lds_limit = 65536;
  size_t device_bytes = 0;
  std::vector<void*> owned;

  double* state[2] = {nullptr, nullptr};
  int cur = 0;               // state[cur] is the committed state
  ttk::UpdatePlan plan[2];        // plan[p] reads state[p], writes state[p ^ 1], then prepares the next update
  ttk::UpdatePlan sweep0[2];      // sweep0[p]: the preparation alone, from state[p] (creation, set_state)
  double* work = nullptr;
  double* Rbuf = nullptr;
  int64_t* trace = nullptr;  // 2 stamps per chain op (TT_FLAG_PROFILE_OPS)
  int64_t trace_len = 0;
  int traced_plan = -1;      // plan of the last traced push
  int wall_khz = 100000;
  std::vector<double*> B;    // B[k] for k = kstar..m-1
  float* B32 = nullptr;
  double* Z = nullptr;
  std::vector<double*> Zk;   // Zk[k] for k = 1..kstar-1
  std::vector<double*> A;    // A[k] for k = 3..kstar+1
  float* A32 = nullptr;
  double* Gt = nullptr;
  double* Y[2] = {nullptr, nullptr};
  double* qrwork = nullptr;
  // the "w/o Ortho" ablation: GB[k] = B_k B_k^T and GBi[k] = (B_k B_k^T)^+
  // (k = 1..m), a J x J Gram matrix and its inverse, scratch, and G~ R_k
  std::vector<double*> GB, GBi;
  double* gram_j = nullptr;
  double* gram_ji = nullptr;
  double* gram_tmp = nullptr;
  double* gram_g = nullptr;
  float* ws = nullptr;       // pass 1 workspace
  float* ws2 = nullptr;      // pass 2 workspace (BF16 contractions only)
  int* flag = nullptr;
  int* rejected = nullptr;
  int64_t* tdev = nullptr;
  double* hist = nullptr;
  int64_t hist_cap = 0;
  double* recon[2] = {nullptr, nullptr};
  void* stage = nullptr;
  size_t stage_bytes = 0;
  ttk::Pass1Plan p1;
  ttk::PassBPlan p1b, p2b;   // BF16 contractions
  int rejected_seen = 0;
  int64_t pushes = 0;
  int64_t hist_t0 = 0;       // update count when the history ring was (re)started
  // serving: the server the stream is registered with (its lanes, not the
  // stream's own HIP stream, then run its updates) and the completion event of
  // the last wave a lane launched for it (owned by the lane)
  struct tt_server* server = nullptr;
  int32_t server_id = -1;
  hipEvent_t ext_done = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evcopy = nullptr;
  hipEvent_t evcommit = nullptr;  // recorded when the last pushed update has committed
  // TT_FLAG_PROFILE_OPS: per pass, before it, after its contraction kernel,
  // after its reduction (pass 1: 0, 1, 2; pass 2: 3, 4, 5)
  hipEvent_t evpass[6] = {};
  bool timed = false;

  double* g_of(double* st) const { return st + coff[m + 1]; }
  double* G_of(double* st, int k) const { return st + coff[k]; }
  double* master() const { return state[cur]; }
};

namespace ttk {

// Live handles of every kind: a handle is checked against this registry
// before it is dereferenced, so a destroyed (freed) handle is rejected rather
// than read.
enum HandleKind { kHandleStream = 1, kHandleBatch = 2, kHandleServer = 3 };
void handle_register(const void* p, int kind);
void handle_unregister(const void* p);
bool handle_live(const void* p, int kind);

inline bool stream_valid(const tt_stream* s) {
  return s != nullptr && handle_live(s, kHandleStream) && s->magic == kStreamMagic;
}

// Waits for all work that may read or write the stream's state: its own HIP
// stream and, when a server runs its updates, the last wave a lane launched
// for it.
hipError_t stream_quiesce(const tt_stream* s);

// A registered stream is being destroyed: the server drops its queued
// requests and refuses further ones for that id (its lanes' waves that used
// the stream have completed: the caller quiesced it).
void server_forget(struct tt_server* sv, int32_t id);

// Records msg as the calling thread's last error and returns st (std::string form).
inline tt_status fail_msg(tt_status st, const std::string& msg) { return set_error(st, msg.c_str()); }

}  // namespace ttk

#define TT_HIP_RT(call)                                                                          \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return ttk::fail_msg(TT_ERR_DEVICE, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
  } while (0)
