// gfx950 element-wise and data-movement kernels of the spectral Poisson
// solver: parity-blocked permutation, transpose, finalization, fill.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

template <typename T>
__global__ void k_finalize(const T *__restrict__ x, const double *__restrict__ ab,
                           const double *__restrict__ tab, double *__restrict__ out, int mode,
                           const double *__restrict__ sinv, int64_t n, int64_t npad, int64_t mp0,
                           int64_t mstride, int64_t ncmax) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (col >= npad) return;
  const int s = r >= mp0 ? 1 : 0;
  const int64_t k = r - (s ? mp0 : 0);
  const int64_t c = k / kChunk;
  const double *tp = tab + (int64_t)s * kNTab * mstride;
  const double *e = ab + (((int64_t)s * ncmax + c) * npad + col) * 2;
  const double v = (double)x[r * npad + col] + e[0] * tp[T_BF2 * mstride + k] +
                   e[1] * tp[T_BK2 * mstride + k];
  if (mode == 0) {
    out[r * npad + col] = v;
    return;
  }
  if (mode == 2) {
    out[r * npad + col] += v;
    return;
  }
  const int t = col >= mp0 ? 1 : 0;
  const int64_t kc = col - (t ? mp0 : 0);
  const int64_t i = 2 * k + s, j = 2 * kc + t;
  if (i >= n || j >= n) return;
  out[i * n + j] = sinv ? v * sinv[i] * sinv[j] : v;
}

__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ G,
                                                  const double *__restrict__ Y,
                                                  const double *__restrict__ dv,
                                                  const double *__restrict__ ev,
                                                  float *__restrict__ r, float *__restrict__ rT,
                                                  int64_t npad) {
  __shared__ float tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int64_t q = c0 + tx;
  const double dq = dv[q], eq = ev[q], eql = q > 0 ? ev[q - 1] : 0.0;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t i = r0 + rr;
    double res = G[i * npad + q];
    if (Y != nullptr) {
      const double *y = Y + i * npad + q;
      const double yc = y[0];
      const double yu = i > 0 ? y[-npad] : 0.0, yd = i + 1 < npad ? y[npad] : 0.0;
      const double yl = q > 0 ? y[-1] : 0.0, yr = q + 1 < npad ? y[1] : 0.0;
      const double eil = i > 0 ? ev[i - 1] : 0.0;
      res -= (dv[i] + dq) * yc + eil * yu + ev[i] * yd + eql * yl + eq * yr;
    }
    r[i * npad + q] = (float)res;
    tile[rr][tx] = (float)res;
  }
  __syncthreads();
  for (int rr = ty; rr < 64; rr += 4) rT[(c0 + rr) * npad + r0 + tx] = tile[tx][rr];
}

__global__ void k_permute_out(const double *__restrict__ src, double *__restrict__ dst, int64_t n,
                              int64_t npad, int64_t mp0, const double *__restrict__ sinv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= n) return;
  const int64_t r = (i & 1) * mp0 + (i >> 1), q = (j & 1) * mp0 + (j >> 1);
  double v = src[r * npad + q];
  if (sinv) v *= sinv[i] * sinv[j];
  dst[i * n + j] = v;
}

__global__ void k_permute_in(const double *__restrict__ src, double *__restrict__ dst, int64_t n,
                             int64_t npad, int64_t mp0, const double *__restrict__ sinv) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (q >= npad) return;
  const int s = r >= mp0 ? 1 : 0, t = q >= mp0 ? 1 : 0;
  const int64_t i = 2 * (r - (s ? mp0 : 0)) + s, j = 2 * (q - (t ? mp0 : 0)) + t;
  double v = 0.0;
  if (i < n && j < n) {
    v = src[i * n + j];
    if (sinv) v *= sinv[i] * sinv[j];
  }
  dst[r * npad + q] = v;
}

__global__ __launch_bounds__(256) void k_transpose(const double *__restrict__ src,
                                                   double *__restrict__ dst, int64_t npad) {
  __shared__ double tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  for (int i = ty; i < 64; i += 4) tile[i][tx] = src[(r0 + i) * npad + c0 + tx];
  __syncthreads();
  for (int i = ty; i < 64; i += 4) dst[(c0 + i) * npad + r0 + tx] = tile[tx][i];
}

__global__ void k_fill(double *__restrict__ dst, int64_t count, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = v;
}

}  // namespace

template <typename T>
hipError_t launch_finalize(const T *x, const double *ab, const double *tab, double *out, int mode,
                           const double *sinv, int64_t n, int64_t npad, int64_t mp0,
                           int64_t mstride, int64_t ncmax, hipStream_t st) {
  dim3 grid((unsigned)((npad + 255) / 256), (unsigned)npad);
  hipLaunchKernelGGL(k_finalize<T>, grid, dim3(256), 0, st, x, ab, tab, out, mode, sinv, n, npad,
                     mp0, mstride, ncmax);
  return hipGetLastError();
}
template hipError_t launch_finalize<double>(const double *, const double *, const double *, double *,
                                            int, const double *, int64_t, int64_t, int64_t, int64_t,
                                            int64_t, hipStream_t);
template hipError_t launch_finalize<float>(const float *, const double *, const double *, double *,
                                           int, const double *, int64_t, int64_t, int64_t, int64_t,
                                           int64_t, hipStream_t);

hipError_t launch_residual(const double *G, const double *Y, const double *dv, const double *ev,
                           float *r, float *rT, int64_t npad, hipStream_t st) {
  if (npad % 64 != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(npad / 64), (unsigned)(npad / 64));
  hipLaunchKernelGGL(k_residual, grid, dim3(256), 0, st, G, Y, dv, ev, r, rT, npad);
  return hipGetLastError();
}

hipError_t launch_permute_in(const double *src, double *dst, int64_t n, int64_t npad, int64_t mp0,
                             hipStream_t st, const double *sinv) {
  dim3 grid((unsigned)((npad + 255) / 256), (unsigned)npad);
  hipLaunchKernelGGL(k_permute_in, grid, dim3(256), 0, st, src, dst, n, npad, mp0, sinv);
  return hipGetLastError();
}

hipError_t launch_permute_out(const double *src, double *dst, int64_t n, int64_t npad, int64_t mp0,
                              const double *sinv, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL(k_permute_out, grid, dim3(256), 0, st, src, dst, n, npad, mp0, sinv);
  return hipGetLastError();
}

hipError_t launch_transpose(const double *src, double *dst, int64_t npad, hipStream_t st) {
  if (npad % 64 != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(npad / 64), (unsigned)(npad / 64));
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, st, src, dst, npad);
  return hipGetLastError();
}

hipError_t launch_fill(double *dst, int64_t count, double v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, dst, count,
                     v);
  return hipGetLastError();
}

}  // namespace fps
