// Measurement aid: a pure streaming pass, c = a + b over n doubles (two
// reads and one write per element, 16-byte accesses), whose rate on arrays
// far larger than the last-level cache is the HBM rate a kernel of the
// sweeps' access pattern can reach.  Not part of the solver.
#include <hip/hip_runtime.h>

#include "launch_limits.hpp"
#include "solver.hpp"

namespace {

typedef double dbl2 __attribute__((ext_vector_type(2)));

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 4;  // 16-byte elements per thread and array

// Workgroup b covers the 16-byte elements [b T U, (b + 1) T U) of each array
// (T threads, U per thread, consecutive threads on consecutive elements);
// the loads of a and b are non-temporal, as the sweeps' G loads are.
__global__ __launch_bounds__(kProbeThreads) void k_stream_sum(const dbl2 *__restrict__ a,
                                                              const dbl2 *__restrict__ b,
                                                              dbl2 *__restrict__ c, int64_t n2) {
  const int64_t base = (int64_t)blockIdx.x * (kProbeThreads * kProbeUnroll) + threadIdx.x;
  dbl2 x[kProbeUnroll], y[kProbeUnroll];
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) {
    const int64_t i = base + (int64_t)u * kProbeThreads;
    const int64_t k = i < n2 ? i : n2 - 1;
    x[u] = __builtin_nontemporal_load(a + k);
    y[u] = __builtin_nontemporal_load(b + k);
  }
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) {
    const int64_t i = base + (int64_t)u * kProbeThreads;
    if (i < n2) c[i] = x[u] + y[u];
  }
}

// The last element of an odd-length array.
__global__ void k_stream_tail(const double *a, const double *b, double *c, int64_t n) {
  if (threadIdx.x == 0) c[n - 1] = a[n - 1] + b[n - 1];
}

}  // namespace

extern "C" fps_status fps_probe_stream(const double *a, const double *b, double *c, int64_t n,
                                       void *stream) {
  if (n < 0) return fps::detail::fail(FPS_E_ARG, "n must be >= 0");
  if (n == 0) return FPS_OK;
  if (a == nullptr || b == nullptr || c == nullptr)
    return fps::detail::fail(FPS_E_ARG, "null array");
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) % 16 != 0)
    return fps::detail::fail(FPS_E_ARG, "arrays must be 16-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  const int64_t n2 = n / 2;
  if (n2 > 0) {
    const int64_t per = (int64_t)kProbeThreads * kProbeUnroll;
    const int64_t grid = (n2 + per - 1) / per;
    if (grid > fps::max_workgroups_1d(kProbeThreads)) return fps::detail::fail(FPS_E_UNSUPPORTED, "array too long");
    hipLaunchKernelGGL(k_stream_sum, dim3((unsigned)grid), dim3(kProbeThreads), 0, st,
                       (const dbl2 *)a, (const dbl2 *)b, (dbl2 *)c, n2);
    FPS_HIP(hipGetLastError());
  }
  if (n % 2 != 0) {
    hipLaunchKernelGGL(k_stream_tail, dim3(1), dim3(64), 0, st, a, b, c, n);
    FPS_HIP(hipGetLastError());
  }
  return FPS_OK;
}
