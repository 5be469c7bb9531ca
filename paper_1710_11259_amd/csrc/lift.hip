// gfx950 kernels of the nonhomogeneous Dirichlet lift (Sec. 6.1): the
// solution is u = u0 + u_bc with u_bc the transfinite interpolant of the four
// boundary traces,
//   u_bc = (1-s)/2 L(t) + (1+s)/2 R(t) + (1-t)/2 B(s) + (1+t)/2 T(s)
//          - (bilinear interpolant of the corner values B(-1), B(1), T(-1), T(1)),
// and u0 the zero-data solution for f - Lap u_bc.  Because u_bc is linear in
// s in its L, R terms and linear in t in its B, T terms,
//   Lap u_bc = sx2 [(1-t)/2 B''(s) + (1+t)/2 T''(s)]
//            + sy2 [(1-s)/2 L''(t) + (1+s)/2 R''(t)],
// whose C~ x C~ coefficients live in rows 0, 1 and columns 0, 1 only (a
// linear function has C~ coefficients at degrees 0 and 1).  All work here is
// O(n) except the C~ map of the four second derivatives (4 matrix-vector
// products with the upper-triangular Chebyshev -> C~ blocks).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

constexpr int kD2Threads = 256;

// Chebyshev derivative by same-parity suffix sums: for c of length N,
//   d_j = (2 / kappa_j) sum_{m > j, m - j odd} m c_m,  j < N - 1,
// kappa_0 = 2, kappa_j = 1 otherwise (the coefficient form of the
// derivative of sum c_m T_m; the classical backward recurrence
// d_{m-1} = d_{m+1} + 2 m c_m summed out).  Each thread owns a contiguous
// segment; segment totals per parity are suffix-scanned across the
// workgroup in LDS.  Ends with a barrier (d visible to the workgroup).
__device__ void cheb_derivative(const double *c, double *d, int64_t N, double *lds) {
  const int t = threadIdx.x;
  const int64_t seg = (N + kD2Threads - 1) / kD2Threads;
  const int64_t lo = t * seg < N ? t * seg : N;
  const int64_t hi = lo + seg < N ? lo + seg : N;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t m = lo; m < hi; ++m) {
    const double a = (double)m * c[m];
    if (m & 1)
      s1 += a;
    else
      s0 += a;
  }
  lds[t] = s0;
  lds[kD2Threads + t] = s1;
  __syncthreads();
  if (t < 2) {  // exclusive suffix over the segments, one parity per thread
    double run = 0.0;
    for (int u = kD2Threads - 1; u >= 0; --u) {
      const double v = lds[t * kD2Threads + u];
      lds[t * kD2Threads + u] = run;
      run += v;
    }
  }
  __syncthreads();
  double run0 = lds[t], run1 = lds[kD2Threads + t];
  for (int64_t m = hi - 1; m >= lo; --m) {
    const double a = (double)m * c[m];
    double Q;
    if (m & 1) {
      run1 += a;
      Q = run1;
    } else {
      run0 += a;
      Q = run0;
    }
    if (m >= 1) d[m - 1] = (m == 1 ? 1.0 : 2.0) * Q;
  }
  __syncthreads();
}

// One workgroup per trace (L, R, B, T): first derivative into d1 [4][N],
// second derivative into d2 [4][n], and the trace's values at -1 and +1
// into corner[2 tr], corner[2 tr + 1].
__global__ __launch_bounds__(kD2Threads) void k_bc_d2(const double *__restrict__ bc,
                                                      double *__restrict__ d1,
                                                      double *__restrict__ d2,
                                                      double *__restrict__ corner, int64_t n) {
  __shared__ double lds[2 * kD2Threads];
  const int tr = blockIdx.x, t = threadIdx.x;
  const int64_t N = n + 2;
  const double *c = bc + tr * N;
  cheb_derivative(c, d1 + tr * N, N, lds);
  cheb_derivative(d1 + tr * N, d2 + tr * n, N - 1, lds);
  double vm = 0.0, vp = 0.0;
  for (int64_t k = t; k < N; k += kD2Threads) {
    vp += c[k];
    vm += (k & 1) ? -c[k] : c[k];
  }
  lds[t] = vm;
  lds[kD2Threads + t] = vp;
  __syncthreads();
  for (int h = kD2Threads / 2; h > 0; h >>= 1) {
    if (t < h) {
      lds[t] += lds[t + h];
      lds[kD2Threads + t] += lds[kD2Threads + t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    corner[2 * tr] = lds[0];
    corner[2 * tr + 1] = lds[kD2Threads];
  }
}

// w[X][pos] = (S^-1 R e_X) at the parity-blocked position of natural index
// i = 2k + s: sum over l >= k of Rs_s[k][l] e_X[2l + s] (Rs_s upper
// triangular, row stride mp_s).  One wavefront per output row.
__global__ __launch_bounds__(256) void k_bc_cmap(const double *__restrict__ Rs0,
                                                 const double *__restrict__ Rs1,
                                                 const double *__restrict__ e,
                                                 double *__restrict__ w, int64_t n, int64_t npad,
                                                 int64_t m0, int64_t mp0, int64_t mp1) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;  // uniform per wavefront
  const int s = row < m0 ? 0 : 1;
  const int64_t k = s ? row - m0 : row;
  const int64_t m = s ? n - m0 : m0;
  const double *Rrow = (s ? Rs1 : Rs0) + k * (s ? mp1 : mp0);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int64_t l = k + lane; l < m; l += 64) {
    const double r = Rrow[l];
    const int64_t i = 2 * l + s;
    a0 += r * e[i];
    a1 += r * e[n + i];
    a2 += r * e[2 * n + i];
    a3 += r * e[3 * n + i];
  }
  for (int off = 32; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off, 64);
    a1 += __shfl_xor(a1, off, 64);
    a2 += __shfl_xor(a2, off, 64);
    a3 += __shfl_xor(a3, off, 64);
  }
  if (lane == 0) {
    const int64_t pos = s * mp0 + k;
    w[pos] = a0;
    w[npad + pos] = a1;
    w[2 * npad + pos] = a2;
    w[3 * npad + pos] = a3;
  }
}

__device__ inline int64_t ppos(int64_t i, int64_t mp0) { return (i & 1) * mp0 + (i >> 1); }

// G -= S^-1 C~(Lap u_bc) S^-1 on rows 0, 1 and columns 0, 1 (natural
// indices; G parity-blocked, row stride npad).  One thread per touched
// entry, so the corner entries that collect both terms are not shared.
__global__ void k_bc_rhs(double *__restrict__ G, const double *__restrict__ w, int64_t n,
                         int64_t npad, int64_t mp0, double sx2, double sy2, BcLiftConst k) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n2 = n < 2 ? n : 2;
  if (e >= n2 * n + (n - n2) * n2) return;
  int64_t i, j;
  if (e < n2 * n) {
    i = e / n;
    j = e % n;
  } else {
    const int64_t f = e - n2 * n;
    i = n2 + f / n2;
    j = f % n2;
  }
  const int64_t pi = ppos(i, mp0), pj = ppos(j, mp0);
  double v = 0.0;
  if (i < 2)  // sx2 [(1-t)/2 B'' + (1+t)/2 T'']: B is trace 2, T trace 3
    v += k.sinv[i] * sx2 * (k.am[i] * w[2 * npad + pj] + k.ap[i] * w[3 * npad + pj]);
  if (j < 2)  // sy2 [(1-s)/2 L'' + (1+s)/2 R'']: L is trace 0, R trace 1
    v += k.sinv[j] * sy2 * (w[pi] * k.am[j] + w[npad + pi] * k.ap[j]);
  G[pi * npad + pj] -= v;
}

// U += Chebyshev coefficients of u_bc (natural (n+2) x (n+2), rows <-> t).
// (1 -+ s)/2 has Chebyshev coefficients (1/2, -+1/2).
__global__ void k_bc_out(double *__restrict__ U, const double *__restrict__ bc,
                         const double *__restrict__ corner, int64_t n) {
  const int64_t N = n + 2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 2 * N + (N - 2) * 2) return;
  int64_t j, k;
  if (e < 2 * N) {
    j = e / N;
    k = e % N;
  } else {
    const int64_t f = e - 2 * N;
    j = 2 + f / 2;
    k = f % 2;
  }
  const double hm[2] = {0.5, -0.5}, hp[2] = {0.5, 0.5};
  const double *L = bc, *R = bc + N, *B = bc + 2 * N, *T = bc + 3 * N;
  double v = 0.0;
  if (k < 2) v += L[j] * hm[k] + R[j] * hp[k];
  if (j < 2) v += hm[j] * B[k] + hp[j] * T[k];
  if (j < 2 && k < 2) {
    const double c00 = corner[4], c10 = corner[5], c01 = corner[6], c11 = corner[7];
    v -= hm[j] * hm[k] * c00 + hm[j] * hp[k] * c10 + hp[j] * hm[k] * c01 + hp[j] * hp[k] * c11;
  }
  U[j * N + k] += v;
}

}  // namespace

hipError_t launch_bc_lift_rhs(const double *bc, const double *Rs0, const double *Rs1, double *G,
                              double *scratch, const Layout &L, double sx2, double sy2,
                              const BcLiftConst &k, hipStream_t st) {
  const int64_t n = L.n, N = n + 2;
  double *d1 = scratch, *d2 = d1 + 4 * N, *w = d2 + 4 * n, *corner = w + 4 * L.npad;
  hipLaunchKernelGGL(k_bc_d2, dim3(4), dim3(kD2Threads), 0, st, bc, d1, d2, corner, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bc_cmap, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Rs0, Rs1, d2, w, n,
                     L.npad, L.m[0], L.mp[0], L.mp[1]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t n2 = n < 2 ? n : 2, total = n2 * n + (n - n2) * n2;
  hipLaunchKernelGGL(k_bc_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, G, w, n,
                     L.npad, L.mp[0], sx2, sy2, k);
  return hipGetLastError();
}

hipError_t launch_bc_lift_out(double *U, const double *bc, const double *scratch, int64_t n,
                              int64_t npad, hipStream_t st) {
  const int64_t N = n + 2, total = 2 * N + (N - 2) * 2;
  const double *corner = scratch + 4 * N + 4 * n + 4 * npad;
  hipLaunchKernelGGL(k_bc_out, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, U, bc,
                     corner, n);
  return hipGetLastError();
}

}  // namespace fps
