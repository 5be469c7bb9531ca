// Allocation-free square / rectangle solve: fps_solve with its workspace in
// a fixed device array that the library holds, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ variable.  Its name in host code is a
// host-side stand-in, not a device address, so the device address is looked
// up once per device with hipGetSymbolAddress (with that device current) and
// only that address is ever handed to kernels.  Each GPU holds its own copy
// until the process ends; every call on one GPU shares it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "solver.hpp"

namespace {

constexpr int64_t kScratchBytes = int64_t(64) << 20;  // 64 MiB
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device (looked up on the
// first call per device).
fps_status scratch_ptr(void **out) {
  int dev = -1;
  FPS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fps::detail::fail(FPS_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[dev] == nullptr) {
    void *p = nullptr;
    FPS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return fps::detail::fail(FPS_E_HIP, "scratch symbol has no device address");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return FPS_OK;
}

}  // namespace

extern "C" {

int64_t fps_noalloc_capacity(void) { return kScratchBytes; }

fps_status fps_solve_noalloc(fps_plan *pl, const double *F, double *U, void *stream) {
  using fps::detail::fail;
  if (!fps::detail::valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (pl->dim != 2 || pl->cyl != nullptr)
    return fail(FPS_E_UNSUPPORTED, "the allocation-free solve takes square and rectangle plans only");
  if (pl->ws_bytes > kScratchBytes)
    return fail(FPS_E_UNSUPPORTED, "the plan's workspace (" + std::to_string(pl->ws_bytes) +
                                       " bytes) exceeds the library's static scratch (" +
                                       std::to_string(kScratchBytes) + " bytes)");
  void *ws = nullptr;
  fps_status s = scratch_ptr(&ws);
  if (s != FPS_OK) return s;
  return fps_solve(pl, F, U, ws, stream);
}

}  // extern "C"
