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
// linear function has C~ coefficients at degrees 0 and 1).  The 1-D factors
// S^-1 C~(g'') come from the plan's lift map applied to the traces' Chebyshev
// coefficients (4 matrix-vector products with its parity blocks); all other
// work is O(n).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

constexpr int kCornerThreads = 256;

// One workgroup per trace (L, R, B, T): its values at -1 and +1 into
// corner[2 tr], corner[2 tr + 1].
__global__ __launch_bounds__(kCornerThreads) void k_bc_corner(const double *__restrict__ bc,
                                                              double *__restrict__ corner,
                                                              int64_t n) {
  __shared__ double lds[2 * kCornerThreads];
  const int tr = blockIdx.x, t = threadIdx.x;
  const int64_t N = n + 2;
  const double *c = bc + tr * N;
  double vm = 0.0, vp = 0.0;
  for (int64_t k = t; k < N; k += kCornerThreads) {
    vp += c[k];
    vm += (k & 1) ? -c[k] : c[k];
  }
  lds[t] = vm;
  lds[kCornerThreads + t] = vp;
  __syncthreads();
  for (int h = kCornerThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      lds[t] += lds[t + h];
      lds[kCornerThreads + t] += lds[kCornerThreads + t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    corner[2 * tr] = lds[0];
    corner[2 * tr + 1] = lds[kCornerThreads];
  }
}

// w[X][pos] = S^-1 C~(g_X'') at the parity-blocked position of natural index
// i = 2a + s: sum over b > a of Ms_s[a][b] g_X[2b + s] (Ms_s has row length
// mo_s; T''_k has C~ components only below degree k - 1).  One wavefront per
// output row.
__global__ __launch_bounds__(256) void k_bc_cmap(const double *__restrict__ Ms0,
                                                 const double *__restrict__ Ms1,
                                                 const double *__restrict__ bc,
                                                 double *__restrict__ w, int64_t n, int64_t npad,
                                                 int64_t m0, int64_t mp0, int64_t mo0,
                                                 int64_t mo1) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;  // uniform per wavefront
  const int s = row < m0 ? 0 : 1;
  const int64_t a = s ? row - m0 : row;
  const int64_t mo = s ? mo1 : mo0, N = n + 2;
  const double *Mrow = (s ? Ms1 : Ms0) + a * mo;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int64_t b = a + 1 + lane; b < mo; b += 64) {
    const double m = Mrow[b];
    const int64_t k = 2 * b + s;
    a0 += m * bc[k];
    a1 += m * bc[N + k];
    a2 += m * bc[2 * N + k];
    a3 += m * bc[3 * N + k];
  }
  for (int off = 32; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off, 64);
    a1 += __shfl_xor(a1, off, 64);
    a2 += __shfl_xor(a2, off, 64);
    a3 += __shfl_xor(a3, off, 64);
  }
  if (lane == 0) {
    const int64_t pos = s * mp0 + a;
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

hipError_t launch_bc_lift_rhs(const double *bc, const double *Ms0, const double *Ms1, double *G,
                              double *scratch, const Layout &L, double sx2, double sy2,
                              const BcLiftConst &k, hipStream_t st) {
  const int64_t n = L.n;
  double *w = scratch, *corner = w + 4 * L.npad;
  hipLaunchKernelGGL(k_bc_corner, dim3(4), dim3(kCornerThreads), 0, st, bc, corner, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bc_cmap, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, Ms0, Ms1, bc, w,
                     n, L.npad, L.m[0], L.mp[0], L.mo[0], L.mo[1]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t n2 = n < 2 ? n : 2, total = n2 * n + (n - n2) * n2;
  hipLaunchKernelGGL(k_bc_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, G, w, n,
                     L.npad, L.mp[0], sx2, sy2, k);
  return hipGetLastError();
}

hipError_t launch_bc_lift_out(double *U, const double *bc, const double *scratch, int64_t n,
                              int64_t npad, hipStream_t st) {
  const int64_t N = n + 2, total = 2 * N + (N - 2) * 2;
  const double *corner = scratch + 4 * npad;
  hipLaunchKernelGGL(k_bc_out, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, U, bc,
                     corner, n);
  return hipGetLastError();
}

}  // namespace fps
