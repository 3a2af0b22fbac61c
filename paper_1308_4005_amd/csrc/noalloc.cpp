// mls_evaluate_noalloc: one MLS evaluation (the path of mls_evaluate) for
// callers that cannot allocate device memory.  The plan's workspace lives in
// a file-scope device array of fixed size instead of hipMalloc'd buffers.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress and only that
// address is ever handed to copies, fills and kernels.  Each device holds its
// own copy of the array until the process ends.  All calls on one device
// share it: a call first waits for the caller's stream (so an earlier call's
// kernels on that stream are done before the tables are rewritten), then
// rebuilds every table and clears what must start at zero, as plan creation
// does.  Calls that overlap on one device (other streams, other threads)
// race on the array.
#include <mutex>
#include <string>

#include "mls_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once).
mls_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    mls::set_error("mls_evaluate_noalloc: device index out of range");
    return MLS_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return mls::hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress(scratch)");
    }
    g_ptr[dev] = (unsigned char*)p;
  }
  *out = g_ptr[dev];
  return MLS_OK;
}

}  // namespace

extern "C" mls_status mls_evaluate_noalloc(const mls_params* params, int64_t n, const double* pos, const double* c6,
                                           double* energy, double* forces, double* potential, double* dE_dc6,
                                           void* stream) {
  using namespace mls;
  if (!params) { set_error("mls_evaluate_noalloc: null params"); return MLS_ERR_INVALID_ARG; }
  if (params->mixing != MLS_GEOMETRIC) {
    set_error("mls_evaluate_noalloc: geometric mixing only");
    return MLS_ERR_INVALID_ARG;
  }
  if (n < 0) { set_error("mls_evaluate_noalloc: n < 0"); return MLS_ERR_INVALID_ARG; }
  if (!energy) { set_error("mls_evaluate_noalloc: energy pointer is required"); return MLS_ERR_INVALID_ARG; }
  if (n > 0 && (!pos || !c6)) { set_error("mls_evaluate_noalloc: null pos or c6"); return MLS_ERR_INVALID_ARG; }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  unsigned char* base = nullptr;
  mls_status st = scratch_address(dev, &base);
  if (st != MLS_OK) return st;
  // an earlier call's kernels on this stream still read the array
  e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  mls_plan_s P;
  P.arena = base;
  P.arena_cap = kScratchBytes;
  P.serial = true;
  st = build_plan(*params, n, &P);
  if (st == MLS_ERR_UNSUPPORTED && std::string(mls_last_error()).find("static scratch") != std::string::npos) {
    set_error("mls_evaluate_noalloc: the workspace for n = " + std::to_string(n) +
              " atoms and these grids exceeds the static scratch of " + std::to_string(kScratchBytes) + " bytes");
    return MLS_ERR_UNSUPPORTED;
  }
  if (st != MLS_OK) return st;
  // the plan's buffers and tables are in place: enqueue the evaluation; the
  // host plan struct is not referenced by the enqueued work
  return evaluate_plan(&P, n, pos, c6, energy, forces, potential, dE_dc6, stream);
}
