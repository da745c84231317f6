// C entry points of the individual update kernels (include/tt_kernels.h).
#include "tt_internal.h"
#include "tt_kernels.h"

#include <mutex>
#include <string>

namespace ttk {
hipError_t pass_setup();
}  // namespace ttk

// Workspace of tt_kernel_pass1_noalloc: a fixed device array, one copy per
// GPU, held until the process ends.  Host code never passes its name to a
// kernel: the name is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device (scratch_ptr below).
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) float scratch[kNoAllocScratchBytes / sizeof(float)];


namespace {

tt_status kfail(tt_status st, const char* what, hipError_t e = hipSuccess) {
  std::string msg = std::string("tt_kernel: ") + what;
  if (e != hipSuccess) msg += std::string(": ") + hipGetErrorString(e);
  return ttk::set_error(st, msg.c_str());
}

int device_cus() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus;
}

ttk::Pass1Plan plan_for(int64_t P, int64_t J, int r) { return ttk::pass1_plan(P, J, r, device_cus()); }

// Device address of this device's `scratch`, looked up on the first call per
// device (with that device current) and kept; null if the lookup failed.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

size_t lds_limit() {
  int dev = 0, lds = 65536;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  return (size_t)lds;
}

}  // namespace

extern "C" {

size_t tt_kernel_pass1_workspace(int64_t P, int64_t J, int32_t r) {
  if (P < 1 || J < 1 || r < 1 || r > 64) return 0;
  return plan_for(P, J, r).ws_floats * sizeof(float);
}

tt_status tt_kernel_pass1(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r, const float* B, double* Z,
                          void* workspace, int32_t* nonfinite_flag, void* hip_stream) {
  if (!X || !B || !Z || !workspace || !nonfinite_flag) return kfail(TT_ERR_INVALID_ARG, "null");
  if (P < 1 || J < 1 || r < 1 || r > 64) return kfail(TT_ERR_INVALID_ARG, "size");
  if (ttk::pass_setup() != hipSuccess) return kfail(TT_ERR_DEVICE, "setup");
  const ttk::Pass1Plan pl = plan_for(P, J, r);
  hipError_t e = ttk::pass1(static_cast<hipStream_t>(hip_stream), X, x_dtype, pl, P, J, r, B, Z,
                            static_cast<float*>(workspace), nonfinite_flag);
  return e == hipSuccess ? TT_OK : kfail(TT_ERR_DEVICE, "pass1", e);
}

tt_status tt_kernel_pass1_noalloc(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r, const float* B,
                                  double* Z, int32_t* nonfinite_flag, void* hip_stream) {
  if (!X || !B || !Z || !nonfinite_flag) return kfail(TT_ERR_INVALID_ARG, "null");
  if (P < 1 || J < 1 || r < 1 || r > 64) return kfail(TT_ERR_INVALID_ARG, "size");
  if (x_dtype != TT_F64 && x_dtype != TT_F32 && x_dtype != TT_BF16) return kfail(TT_ERR_INVALID_ARG, "dtype");
  const ttk::Pass1Plan pl = plan_for(P, J, r);
  if (pl.ws_floats * sizeof(float) > kNoAllocScratchBytes)
    return kfail(TT_ERR_UNSUPPORTED, "pass1_noalloc: the partial tiles of this shape exceed the 32 MiB static "
                                     "scratch (tt_kernel_pass1_workspace(P, J, r) > tt_kernel_pass1_noalloc_max())");
  if (ttk::pass_setup() != hipSuccess) return kfail(TT_ERR_DEVICE, "setup");
  void* ws = nullptr;
  hipError_t e = scratch_ptr(&ws);
  if (e != hipSuccess) return kfail(TT_ERR_DEVICE, "pass1_noalloc: hipGetSymbolAddress of the scratch", e);
  e = ttk::pass1(static_cast<hipStream_t>(hip_stream), X, x_dtype, pl, P, J, r, B, Z, static_cast<float*>(ws),
                 nonfinite_flag);
  return e == hipSuccess ? TT_OK : kfail(TT_ERR_DEVICE, "pass1_noalloc", e);
}

size_t tt_kernel_pass1_noalloc_max(void) { return kNoAllocScratchBytes; }

tt_status tt_kernel_pass2(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r, const float* A, double* Y,
                          int32_t* nonfinite_flag, void* hip_stream) {
  if (!X || !A || !Y || !nonfinite_flag) return kfail(TT_ERR_INVALID_ARG, "null");
  if (P < 1 || J < 1 || r < 1 || r > 64) return kfail(TT_ERR_INVALID_ARG, "size");
  if (ttk::pass_setup() != hipSuccess) return kfail(TT_ERR_DEVICE, "setup");
  hipError_t e = ttk::pass2(static_cast<hipStream_t>(hip_stream), X, x_dtype, P, J, r, A, Y, nonfinite_flag);
  return e == hipSuccess ? TT_OK : kfail(TT_ERR_DEVICE, "pass2", e);
}

size_t tt_kernel_pass1_bf16_workspace(int64_t P, int64_t J, int32_t r) {
  if (P < 1 || J < 1 || r < 1 || r > 64) return 0;
  return ttk::pass1b_plan(P, J, r, device_cus()).ws_bytes;
}

tt_status tt_kernel_pass1_bf16(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r, const float* B,
                               double* Z, void* workspace, int32_t* nonfinite_flag, void* hip_stream) {
  if (!X || !B || !Z || !workspace || !nonfinite_flag) return kfail(TT_ERR_INVALID_ARG, "null");
  if (P < 1 || J < 1 || r < 1 || r > 64) return kfail(TT_ERR_INVALID_ARG, "size");
  const ttk::PassBPlan pl = ttk::pass1b_plan(P, J, r, device_cus());
  hipError_t e = ttk::pass1_bf16(static_cast<hipStream_t>(hip_stream), X, x_dtype, pl, P, J, r, B, Z, workspace,
                                 nonfinite_flag);
  return e == hipSuccess ? TT_OK : kfail(TT_ERR_DEVICE, "pass1_bf16", e);
}

size_t tt_kernel_pass2_bf16_workspace(int64_t P, int64_t J, int32_t r) {
  if (P < 1 || J < 1 || r < 1 || r > 64) return 0;
  return ttk::pass2b_plan(P, J, r, device_cus()).ws_bytes;
}

tt_status tt_kernel_pass2_bf16(const void* X, tt_dtype x_dtype, int64_t P, int64_t J, int32_t r, const float* A,
                               double* Y, void* workspace, int32_t* nonfinite_flag, void* hip_stream) {
  if (!X || !A || !Y || !workspace || !nonfinite_flag) return kfail(TT_ERR_INVALID_ARG, "null");
  if (P < 1 || J < 1 || r < 1 || r > 64) return kfail(TT_ERR_INVALID_ARG, "size");
  if (ttk::pass_bf16_setup() != hipSuccess) return kfail(TT_ERR_DEVICE, "setup");
  const ttk::PassBPlan pl = ttk::pass2b_plan(P, J, r, device_cus());
  hipError_t e = ttk::pass2_bf16(static_cast<hipStream_t>(hip_stream), X, x_dtype, pl, P, J, r, A, Y, workspace,
                                 nonfinite_flag);
  return e == hipSuccess ? TT_OK : kfail(TT_ERR_DEVICE, "pass2_bf16", e);
}

tt_status tt_kernel_qr(int32_t m, int32_t n, const double* M, double* Q, double* R, double* workspace,
                       void* hip_stream) {
  if (!M || !Q || !workspace) return kfail(TT_ERR_INVALID_ARG, "null");
  if (n < 1 || m < n) return kfail(TT_ERR_INVALID_ARG, "size");
  ttk::ChainOp op;
  op.type = ttk::kOpQr;
  op.m = m;
  op.n = n;
  op.rho = n;
  op.a = M;
  op.ars = 1;
  op.acs = m;
  op.c = Q;
  op.crs = 1;
  op.ccs = m;
  op.r = R;
  op.aux = workspace;
  op.tol = 64.0 * 2.220446049250313e-16;
  if (!ttk::chain_op_supported(op)) return kfail(TT_ERR_UNSUPPORTED, "more than 256 columns");
  if (ttk::chain_setup(lds_limit()) != hipSuccess) return kfail(TT_ERR_DEVICE, "setup");
  hipError_t e = ttk::chain_run_one(static_cast<hipStream_t>(hip_stream), op);
  return e == hipSuccess ? TT_OK : kfail(TT_ERR_DEVICE, "qr", e);
}

}  // extern "C"
