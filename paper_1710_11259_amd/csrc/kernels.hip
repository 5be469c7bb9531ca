// gfx950 element-wise and data-movement kernels of the spectral Poisson
// solver: parity-blocked permutation, residual, finalization, fill.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

// Entry (r, col) of the final pass (k_finalize's grid: col = x thread
// index, r = row).
template <typename T>
__device__ __forceinline__ void finalize_at(const T *__restrict__ x, const double *__restrict__ ab,
                                            const double *__restrict__ tab, double *__restrict__ out,
                                            int mode, const double *__restrict__ sinv, int64_t n,
                                            int64_t npad, int64_t mp0, int64_t mstride,
                                            int64_t ncmax, int64_t col, int64_t r) {
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

template <typename T>
__global__ void k_finalize(const T *__restrict__ x, const double *__restrict__ ab,
                           const double *__restrict__ tab, double *__restrict__ out, int mode,
                           const double *__restrict__ sinv, int64_t n, int64_t npad, int64_t mp0,
                           int64_t mstride, int64_t ncmax, int64_t r0) {
  finalize_at<T>(x, ab, tab, out, mode, sinv, n, npad, mp0, mstride, ncmax,
                 (int64_t)blockIdx.x * blockDim.x + threadIdx.x, r0 + blockIdx.y);
}

// 64 x 64 tile (column tile bx, row tile by) of the residual; 256 threads.
__device__ __forceinline__ void residual_tile(const double *__restrict__ G,
                                              const double *__restrict__ Y,
                                              const double *__restrict__ dv,
                                              const double *__restrict__ ev,
                                              float *__restrict__ r, float *__restrict__ rT,
                                              int64_t npad, double ax, double ay, int64_t bx,
                                              int64_t by, float (*tile)[65]) {
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t r0 = by * 64, c0 = bx * 64;
  const int64_t q = c0 + tx;
  const double dq = dv[q], eq = ev[q], eql = q > 0 ? ev[q - 1] : 0.0;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t i = r0 + rr;
    double res = G[i * npad + q];
    if (Y != nullptr) {
      const double *y = Y + i * npad + q;
      const double yc = y[0];
      // rows across a parity-block boundary (zero coupling) are not read:
      // the two row-parity blocks may be computed concurrently
      const double eil = i > 0 ? ev[i - 1] : 0.0, ei = ev[i];
      const double yu = eil != 0.0 ? y[-npad] : 0.0, yd = ei != 0.0 ? y[npad] : 0.0;
      const double yl = q > 0 ? y[-1] : 0.0, yr = q + 1 < npad ? y[1] : 0.0;
      res -= ax * (dv[i] * yc + eil * yu + ei * yd) + ay * (dq * yc + eql * yl + eq * yr);
    }
    r[i * npad + q] = (float)res;
    tile[rr][tx] = (float)res;
  }
  if (rT == nullptr) return;  // uniform: no transposed copy wanted
  __syncthreads();
  for (int rr = ty; rr < 64; rr += 4) rT[(c0 + rr) * npad + r0 + tx] = tile[tx][rr];
}

__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ G,
                                                  const double *__restrict__ Y,
                                                  const double *__restrict__ dv,
                                                  const double *__restrict__ ev,
                                                  float *__restrict__ r, float *__restrict__ rT,
                                                  int64_t npad, double ax, double ay, int64_t by0) {
  __shared__ float tile[64][65];
  residual_tile(G, Y, dv, ev, r, rT, npad, ax, ay, blockIdx.x, by0 + blockIdx.y, tile);
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

// Entry (r, q) of the parity-blocked copy of F (k_permute_in's grid: q = x
// thread index, r = row).
__device__ __forceinline__ void permute_in_at(const double *__restrict__ src,
                                              double *__restrict__ dst, int64_t n, int64_t npad,
                                              int64_t mp0, const double *__restrict__ sinv,
                                              int64_t q, int64_t r) {
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

__global__ void k_permute_in(const double *__restrict__ src, double *__restrict__ dst, int64_t n,
                             int64_t npad, int64_t mp0, const double *__restrict__ sinv) {
  permute_in_at(src, dst, n, npad, mp0, sinv, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                blockIdx.y);
}

// --- batched forms: workgroup g works for problem wg_prob[g] -------------

__device__ __forceinline__ intptr_t elem_base(int id, char *ws, const double *in) {
  return id == 1 ? (intptr_t)ws : id == 2 ? (intptr_t)in : 0;
}

__global__ __launch_bounds__(256) void k_permute_in_batch(const ElemDesc *__restrict__ d,
                                                          const int *__restrict__ wg_prob,
                                                          const double *in, char *ws) {
  const int g = blockIdx.x;
  const ElemDesc &e = d[__builtin_amdgcn_readfirstlane(wg_prob[g])];
  const int local = g - e.wg_start;
  const double *src = (const double *)(elem_base(e.sbase, ws, in) + e.src);
  double *dst = (double *)(elem_base(e.dbase, ws, in) + e.dst);
  permute_in_at(src, dst, e.n, e.npad, e.mp0, nullptr,
                (int64_t)(local % e.nbx) * 256 + threadIdx.x, local / e.nbx);
}


__global__ __launch_bounds__(256) void k_residual_batch(const ElemDesc *__restrict__ d,
                                                        const int *__restrict__ wg_prob,
                                                        int with_y, char *ws) {
  __shared__ float tile[64][65];
  const int g = blockIdx.x;
  const ElemDesc &e = d[__builtin_amdgcn_readfirstlane(wg_prob[g])];
  const int local = g - e.wg_start;
  float *r = (float *)(ws + e.dst);
  residual_tile((const double *)(ws + e.src), with_y ? (const double *)(ws + e.ab) : nullptr, e.tab,
                e.ev, r, nullptr, e.npad, 1.0, 1.0, local % e.nbx, local / e.nbx, tile);
}

template <typename T>
__global__ __launch_bounds__(256) void k_finalize_batch(const ElemDesc *__restrict__ d,
                                                        const int *__restrict__ wg_prob, int mode,
                                                        char *ws) {
  const int g = blockIdx.x;
  const ElemDesc &e = d[__builtin_amdgcn_readfirstlane(wg_prob[g])];
  const int local = g - e.wg_start;
  const T *x = (const T *)(elem_base(e.sbase, ws, nullptr) + e.src);
  double *out = (double *)(elem_base(e.dbase, ws, nullptr) + e.dst);
  finalize_at<T>(x, (const double *)(ws + e.ab), e.tab, out, mode, nullptr, e.n, e.npad, e.mp0,
                 e.mstride, e.ncmax, (int64_t)(local % e.nbx) * 256 + threadIdx.x, local / e.nbx);
}

__global__ void k_fill(double *__restrict__ dst, int64_t count, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = v;
}

// --- cube ----------------------------------------------------------------

__device__ __forceinline__ int64_t pb_index(int64_t i, int64_t mb0) {
  return (i & 1) * mb0 + (i >> 1);
}

// natural n^3 -> parity-blocked npad^3 (zero padding)
__global__ void k_permute3_in(const double *__restrict__ src, double *__restrict__ dst, int64_t n,
                              int64_t npad, int64_t mp0) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ry = blockIdx.y, rz = blockIdx.z;
  if (q >= npad) return;
  auto nat = [&](int64_t r) {
    const int s = r >= mp0 ? 1 : 0;
    return 2 * (r - (s ? mp0 : 0)) + s;
  };
  const int64_t ix = nat(q), iy = nat(ry), iz = nat(rz);
  double v = 0.0;
  if (ix < n && iy < n && iz < n) v = src[(iz * n + iy) * n + ix];
  dst[(rz * npad + ry) * npad + q] = v;
}

// parity-blocked [.][.][ld] (parity-1 block at mb0 on every axis, row
// length ld, plane ld * ld) -> natural N^3, times sinv_i sinv_j sinv_k when
// sinv is non-null.
// A workgroup covers 256 consecutive elements of one output plane (so a
// plane of (n + 2)^2 keeps every lane busy but the last workgroup's).
__global__ void k_permute3_out(const double *__restrict__ src, double *__restrict__ dst, int64_t N,
                               int64_t ld, int64_t mb0, const double *__restrict__ sinv) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x, n32 = (uint32_t)N;
  if (i >= n32 * n32) return;
  const int64_t iy = i / n32, ix = i - (uint32_t)iy * n32, iz = blockIdx.y;
  double v = src[(pb_index(iz, mb0) * ld + pb_index(iy, mb0)) * ld + pb_index(ix, mb0)];
  if (sinv) v *= sinv[iz] * sinv[iy] * sinv[ix];
  dst[(iz * N + iy) * N + ix] = v;
}

// After a z-fiber sweep (chains = the npad^2 (y, x) columns, positions z):
// R = x + chunk carries, written as R[z][y][x] and, per z-slice, R^T[z][x][y].
__global__ __launch_bounds__(256) void k_cube_zfinal(const double *__restrict__ x,
                                                     const double *__restrict__ ab,
                                                     const double *__restrict__ tab,
                                                     double *__restrict__ R,
                                                     double *__restrict__ RT, int64_t npad,
                                                     int64_t mp0, int64_t mstride,
                                                     int64_t ncmax) {
  __shared__ double tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t z = blockIdx.z;
  const int64_t y0 = (int64_t)blockIdx.y * 64, x0 = (int64_t)blockIdx.x * 64;
  const int s = z >= mp0 ? 1 : 0;
  const int64_t k = z - (s ? mp0 : 0), c = k / kChunk;
  const double *tp = tab + (int64_t)s * kNTab * mstride;
  const double bf = tp[T_BF2 * mstride + k], bk = tp[T_BK2 * mstride + k];
  const int64_t plane = npad * npad;
  const double *e = ab + ((int64_t)s * ncmax + c) * plane * 2;
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t col = (y0 + rr) * npad + x0 + tx;
    const double v = x[z * plane + col] + e[2 * col] * bf + e[2 * col + 1] * bk;
    R[z * plane + col] = v;
    tile[rr][tx] = v;
  }
  if (RT == nullptr) return;  // uniform: no transposed copy wanted
  __syncthreads();
  for (int rr = ty; rr < 64; rr += 4) RT[z * plane + (x0 + rr) * npad + y0 + tx] = tile[tx][rr];
}

// Per-slice finalization (chains = x columns, positions y) with the table
// of slice z; slices without a table are cleared.
template <typename T>
__global__ void k_slice_final(const T *__restrict__ x, const double *__restrict__ ab,
                              const double *const *__restrict__ tabs, double *__restrict__ out,
                              double scale, int add, int64_t npad, int64_t mp0, int64_t mstride,
                              int64_t ncmax) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t y = blockIdx.y, z = blockIdx.z;
  if (q >= npad) return;
  const int64_t i = (z * npad + y) * npad + q;
  const double *tab = tabs[z];
  if (tab == nullptr) {
    if (!add) out[i] = 0.0;
    return;
  }
  const int s = y >= mp0 ? 1 : 0;
  const int64_t k = y - (s ? mp0 : 0), c = k / kChunk;
  const double *tp = tab + (int64_t)s * kNTab * mstride;
  const double *e = ab + z * (2 * ncmax * npad * 2) + (((int64_t)s * ncmax + c) * npad + q) * 2;
  const double v =
      scale * ((double)x[i] + e[0] * tp[T_BF2 * mstride + k] + e[1] * tp[T_BK2 * mstride + k]);
  if (add)
    out[i] += v;
  else
    out[i] = v;
}

// Residual of the slice equations of the z-eigenbasis cube, negated:
// q_z = G_z + A~ Y_z A~ + mu_z (A~ Y_z + Y_z A~) on every slice z (Y null:
// q = G), in FP64, stored in float.  A~ acts along each parity block as the
// tridiagonal stencil (dv, ev) of launch_residual.  Each thread walks 16
// rows of one column keeping the row-direction products of three
// consecutive rows, so A~ (Y A~) needs no second pass; 256 threads = 64
// columns x 4 row groups of a 64 x 64 tile.
__global__ __launch_bounds__(256) void k_zeig_residual(const double *__restrict__ G,
                                                       const double *__restrict__ Y,
                                                       const double *__restrict__ dv,
                                                       const double *__restrict__ ev,
                                                       const double *__restrict__ mu,
                                                       float *__restrict__ q, int64_t npad) {
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t z = blockIdx.z;
  const int64_t j = (int64_t)blockIdx.x * 64 + tx;
  const int64_t i0 = (int64_t)blockIdx.y * 64 + ty * 16;
  const int64_t so = z * npad * npad;
  const double *Gz = G + so;
  float *qz = q + so;
  if (Y == nullptr) {
    for (int64_t i = i0; i < i0 + 16; ++i) qz[i * npad + j] = (float)Gz[i * npad + j];
    return;
  }
  const double *Yz = Y + so;
  const double m = mu[z];
  const double dj = dv[j], ej = ev[j], ejl = j > 0 ? ev[j - 1] : 0.0;
  // y(i) and (Y A~)(i) at column j; rows outside [0, npad) are zero
  auto yrow = [&](int64_t i, double *yv, double *ya) {
    if (i < 0 || i >= npad) {
      *yv = 0.0;
      *ya = 0.0;
      return;
    }
    const double *r = Yz + i * npad + j;
    const double yc = r[0];
    const double yl = j > 0 ? r[-1] : 0.0, yr = j + 1 < npad ? r[1] : 0.0;
    *yv = yc;
    *ya = dj * yc + ejl * yl + ej * yr;
  };
  double ym, yam, y0, ya0, yp, yap;
  yrow(i0 - 1, &ym, &yam);
  yrow(i0, &y0, &ya0);
  for (int64_t i = i0; i < i0 + 16; ++i) {
    yrow(i + 1, &yp, &yap);
    const double di = dv[i], ei = ev[i], eil = i > 0 ? ev[i - 1] : 0.0;
    const double ay = di * y0 + eil * ym + ei * yp;      // (A~ Y)(i, j)
    const double aya = di * ya0 + eil * yam + ei * yap;  // (A~ Y A~)(i, j)
    qz[i * npad + j] = (float)(Gz[i * npad + j] + aya + m * (ay + ya0));
    ym = y0;
    yam = ya0;
    y0 = yp;
    ya0 = yap;
  }
}

// After a solve along the rows of every slice that left x (float, chunk
// carries pending in ab with the tables tab, shared by the slices): v = x +
// carries, stored as outT[z][i][j] = v and out[z][j][i] = v (float) through
// a 64 x 64 LDS tile.
__global__ __launch_bounds__(256) void k_slice_xfinal(const float *__restrict__ x,
                                                      const double *__restrict__ ab,
                                                      const double *__restrict__ tab,
                                                      float *__restrict__ outT,
                                                      float *__restrict__ out, int64_t npad,
                                                      int64_t mp0, int64_t mstride, int64_t ncmax) {
  __shared__ float tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t z = blockIdx.z, r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int64_t so = z * npad * npad;
  const double *abz = ab + z * (2 * ncmax * npad * 2);
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t y = r0 + rr, col = c0 + tx;
    const int s = y >= mp0 ? 1 : 0;
    const int64_t k = y - (s ? mp0 : 0), c = k / kChunk;
    const double *tp = tab + (int64_t)s * kNTab * mstride;
    const double *e = abz + (((int64_t)s * ncmax + c) * npad + col) * 2;
    const float v = (float)((double)x[so + y * npad + col] + e[0] * tp[T_BF2 * mstride + k] +
                            e[1] * tp[T_BK2 * mstride + k]);
    outT[so + y * npad + col] = v;
    tile[rr][tx] = v;
  }
  __syncthreads();
  for (int rr = ty; rr < 64; rr += 4) out[so + (c0 + rr) * npad + r0 + tx] = tile[tx][rr];
}

// After the last inner sweep on every z-slice (chains = x columns, positions
// y): Y = x + chunk carries; out = cy Y + cr R + cb B (R, B may be null when
// their coefficient is 0).
__global__ void k_cube_ifinal(const double *__restrict__ x, const double *__restrict__ ab,
                              const double *__restrict__ tab, const double *__restrict__ R,
                              const double *__restrict__ B, double *__restrict__ out, double cy,
                              double cr, double cb, int64_t npad, int64_t mp0, int64_t mstride,
                              int64_t ncmax) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t y = blockIdx.y, z = blockIdx.z;
  if (q >= npad) return;
  const int s = y >= mp0 ? 1 : 0;
  const int64_t k = y - (s ? mp0 : 0), c = k / kChunk;
  const double *tp = tab + (int64_t)s * kNTab * mstride;
  const int64_t i = (z * npad + y) * npad + q;
  double v = x[i];
  if (ab) {  // null: x is complete (no chunk carries left)
    const double *e = ab + z * (2 * ncmax * npad * 2) + (((int64_t)s * ncmax + c) * npad + q) * 2;
    v = x[i] + e[0] * tp[T_BF2 * mstride + k] + e[1] * tp[T_BK2 * mstride + k];
  }
  v = cy * v;
  if (R) v += cr * R[i];
  if (B) v += cb * B[i];
  out[i] = v;
}

}  // namespace

hipError_t launch_permute3_in(const double *src, double *dst, int64_t n, int64_t npad, int64_t mp0,
                              hipStream_t st) {
  dim3 grid((unsigned)((npad + 255) / 256), (unsigned)npad, (unsigned)npad);
  hipLaunchKernelGGL(k_permute3_in, grid, dim3(256), 0, st, src, dst, n, npad, mp0);
  return hipGetLastError();
}

hipError_t launch_permute3_out(const double *src, double *dst, int64_t N, int64_t ld, int64_t mb0,
                               const double *sinv, hipStream_t st) {
  if (N > 46340) return hipErrorInvalidValue;  // a plane's index fits 32 bits
  dim3 grid((unsigned)((N * N + 255) / 256), (unsigned)N);
  hipLaunchKernelGGL(k_permute3_out, grid, dim3(256), 0, st, src, dst, N, ld, mb0, sinv);
  return hipGetLastError();
}

hipError_t launch_cube_zfinal(const double *x, const double *ab, const double *tab, double *R,
                              double *RT, int64_t npad, int64_t mp0, int64_t mstride,
                              int64_t ncmax, hipStream_t st) {
  if (npad % 64 != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(npad / 64), (unsigned)(npad / 64), (unsigned)npad);
  hipLaunchKernelGGL(k_cube_zfinal, grid, dim3(256), 0, st, x, ab, tab, R, RT, npad, mp0, mstride,
                     ncmax);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_slice_final(const T *x, const double *ab, const double *const *tabs, double *out,
                              double scale, int add, int64_t npad, int64_t mp0, int64_t mstride,
                              int64_t ncmax, hipStream_t st) {
  dim3 grid((unsigned)((npad + 255) / 256), (unsigned)npad, (unsigned)npad);
  hipLaunchKernelGGL(k_slice_final<T>, grid, dim3(256), 0, st, x, ab, tabs, out, scale, add, npad,
                     mp0, mstride, ncmax);
  return hipGetLastError();
}
template hipError_t launch_slice_final<double>(const double *, const double *, const double *const *,
                                               double *, double, int, int64_t, int64_t, int64_t,
                                               int64_t, hipStream_t);
template hipError_t launch_slice_final<float>(const float *, const double *, const double *const *,
                                              double *, double, int, int64_t, int64_t, int64_t,
                                              int64_t, hipStream_t);

hipError_t launch_zeig_residual(const double *G, const double *Y, const double *dv, const double *ev,
                                const double *mu, float *q, int64_t npad, int64_t nslices,
                                hipStream_t st) {
  if (npad % 64 != 0 || nslices <= 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(npad / 64), (unsigned)(npad / 64), (unsigned)nslices);
  hipLaunchKernelGGL(k_zeig_residual, grid, dim3(256), 0, st, G, Y, dv, ev, mu, q, npad);
  return hipGetLastError();
}

hipError_t launch_slice_xfinal(const float *x, const double *ab, const double *tab, float *outT,
                               float *out, int64_t npad, int64_t mp0, int64_t mstride,
                               int64_t ncmax, int64_t nslices, hipStream_t st) {
  if (npad % 64 != 0 || nslices <= 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(npad / 64), (unsigned)(npad / 64), (unsigned)nslices);
  hipLaunchKernelGGL(k_slice_xfinal, grid, dim3(256), 0, st, x, ab, tab, outT, out, npad, mp0,
                     mstride, ncmax);
  return hipGetLastError();
}

hipError_t launch_cube_ifinal(const double *x, const double *ab, const double *tab,
                              const double *R, const double *B, double *out, double cy, double cr,
                              double cb, int64_t npad, int64_t mp0, int64_t mstride, int64_t ncmax,
                              hipStream_t st) {
  dim3 grid((unsigned)((npad + 255) / 256), (unsigned)npad, (unsigned)npad);
  hipLaunchKernelGGL(k_cube_ifinal, grid, dim3(256), 0, st, x, ab, tab, R, B, out, cy, cr, cb,
                     npad, mp0, mstride, ncmax);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const T *x, const double *ab, const double *tab, double *out, int mode,
                           const double *sinv, int64_t n, int64_t npad, int64_t mp0,
                           int64_t mstride, int64_t ncmax, hipStream_t st, int64_t r0, int64_t r1) {
  if (r1 < 0) r1 = npad;
  if (r0 < 0 || r1 > npad) return hipErrorInvalidValue;
  if (r0 >= r1) return hipSuccess;
  dim3 grid((unsigned)((npad + 255) / 256), (unsigned)(r1 - r0));
  hipLaunchKernelGGL(k_finalize<T>, grid, dim3(256), 0, st, x, ab, tab, out, mode, sinv, n, npad,
                     mp0, mstride, ncmax, r0);
  return hipGetLastError();
}
template hipError_t launch_finalize<double>(const double *, const double *, const double *, double *,
                                            int, const double *, int64_t, int64_t, int64_t, int64_t,
                                            int64_t, hipStream_t, int64_t, int64_t);
template hipError_t launch_finalize<float>(const float *, const double *, const double *, double *,
                                           int, const double *, int64_t, int64_t, int64_t, int64_t,
                                           int64_t, hipStream_t, int64_t, int64_t);

hipError_t launch_residual(const double *G, const double *Y, const double *dv, const double *ev,
                           float *r, float *rT, int64_t npad, hipStream_t st, double ax,
                           double ay, int64_t r0, int64_t r1) {
  if (r1 < 0) r1 = npad;
  if (npad % 64 != 0 || r0 % 64 != 0 || r1 % 64 != 0 || r0 < 0 || r1 > npad)
    return hipErrorInvalidValue;
  if (r0 >= r1) return hipSuccess;
  if (rT != nullptr && (r0 != 0 || r1 != npad)) return hipErrorInvalidValue;
  dim3 grid((unsigned)(npad / 64), (unsigned)((r1 - r0) / 64));
  hipLaunchKernelGGL(k_residual, grid, dim3(256), 0, st, G, Y, dv, ev, r, rT, npad, ax, ay,
                     r0 / 64);
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

hipError_t launch_permute_in_batch(const ElemDesc *d, const int *wg_prob, int nwg, const double *in,
                                   char *ws, hipStream_t st) {
  if (nwg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_in_batch, dim3((unsigned)nwg), dim3(256), 0, st, d, wg_prob, in, ws);
  return hipGetLastError();
}

hipError_t launch_residual_batch(const ElemDesc *d, const int *wg_prob, int nwg, bool with_y,
                                 char *ws, hipStream_t st) {
  if (nwg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual_batch, dim3((unsigned)nwg), dim3(256), 0, st, d, wg_prob,
                     with_y ? 1 : 0, ws);
  return hipGetLastError();
}

hipError_t launch_finalize_batch(const ElemDesc *d, const int *wg_prob, int nwg, int mode, char *ws,
                                 hipStream_t st, int x_f32) {
  if (nwg <= 0) return hipSuccess;
  if (mode != 0 && mode != 2) return hipErrorInvalidValue;
  if (x_f32)
    hipLaunchKernelGGL(k_finalize_batch<float>, dim3((unsigned)nwg), dim3(256), 0, st, d, wg_prob,
                       mode, ws);
  else
    hipLaunchKernelGGL(k_finalize_batch<double>, dim3((unsigned)nwg), dim3(256), 0, st, d, wg_prob,
                       mode, ws);
  return hipGetLastError();
}

hipError_t launch_fill(double *dst, int64_t count, double v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, dst, count,
                     v);
  return hipGetLastError();
}

}  // namespace fps
