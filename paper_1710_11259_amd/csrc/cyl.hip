// gfx950 kernels of the cylinder solve: the input permutation into the
// parity-blocked per-mode layout and the banded solves in r (one thread per
// |k| and z column, applying the LU factors computed by the plan with
// partial pivoting to the modes k and -k, real and imaginary parts).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

// X0[((slot * 2 + part) * npad + rpos) * npad + zpos] = F[idx][part][i][j]
// (zero at padded positions).  Thread e = ((sp * npad) + rpos) * mp + a
// reads the pair F[..][i][2a], F[..][i][2a + 1] (adjacent lanes read
// adjacent pairs) and writes the even-parity position a and the odd-parity
// position mp + a of row rpos.
__global__ __launch_bounds__(256) void k_cyl_permute_in(const double *__restrict__ F,
                                                        double *__restrict__ X0,
                                                        const int *__restrict__ slot_idx,
                                                        uint32_t n, uint32_t mp, uint32_t total) {
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e >= total) return;
  const uint32_t npad = 2 * mp, m = n / 2;
  const uint32_t a = e % mp, row = e / mp;
  const uint32_t rpos = row % npad, sp = row / npad;
  const uint32_t rs = rpos >= mp ? 1u : 0u, ra = rpos - (rs ? mp : 0u);
  double v0 = 0.0, v1 = 0.0;
  if (ra < m && a < m) {
    const int64_t i = 2 * (int64_t)ra + rs;
    const double *src = F + (((int64_t)slot_idx[sp >> 1] * 2 + (sp & 1)) * n + i) * n + 2 * (int64_t)a;
    v0 = src[0];
    v1 = src[1];
  }
  double *dst = X0 + ((int64_t)sp * npad + rpos) * npad;
  dst[a] = v0;
  dst[mp + a] = v1;
}

// One z column of one |k| group: the banded systems (Q_k + lambda_j P_k)
// yhat = rhs of the group's right-hand sides (up to kCylRhs), sharing the
// factors fac[((kabs * 8 + t) * mp + a) * npad + zpos], t: pivot offset,
// two multipliers, 1/u_aa, four superdiagonal entries of U.  rhs: X0 rows
// of parity rp (column zpos, stride npad), overwritten by the forward
// substitution; yhat: X1 rows of parity wp (zeros beyond m and for padded
// columns).  The factors and right-hand sides of kCylStep consecutive steps
// are loaded before they are used.
constexpr int kCylStep = 8;

__global__ __launch_bounds__(64) void k_cyl_solve(double *__restrict__ X0,
                                                  double *__restrict__ X1,
                                                  const double *__restrict__ fac,
                                                  const CylSolveGroup *__restrict__ grp, int64_t m,
                                                  int64_t mp) {
  const int64_t npad = 2 * mp;
  const int64_t zpos = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (zpos >= npad) return;
  const CylSolveGroup &e = grp[blockIdx.y];
  double *b[kCylRhs], *x[kCylRhs];
  bool use[kCylRhs];
#pragma unroll
  for (int r = 0; r < kCylRhs; ++r) {
    use[r] = e.sp[r] >= 0;
    const int64_t sp = use[r] ? e.sp[r] : e.sp[0];  // unused: recomputed, never stored
    b[r] = X0 + (sp * npad + e.rp * mp) * npad + zpos;
    x[r] = X1 + (sp * npad + e.wp * mp) * npad + zpos;
  }
  const int s = zpos >= mp ? 1 : 0;
  if (zpos - (s ? mp : 0) >= m) {
    for (int64_t a = 0; a < mp; ++a)
#pragma unroll
      for (int r = 0; r < kCylRhs; ++r)
        if (use[r]) x[r][a * npad] = 0.0;
    return;
  }
  const double *f0 = fac + ((int64_t)e.kabs * 8 * mp) * npad + zpos;
  const int64_t fs = mp * npad;  // between factor fields
  double w0[kCylRhs], w1[kCylRhs], w2[kCylRhs];
#pragma unroll
  for (int r = 0; r < kCylRhs; ++r) {
    w0[r] = b[r][0];
    w1[r] = m > 1 ? b[r][npad] : 0.0;
    w2[r] = m > 2 ? b[r][2 * npad] : 0.0;
  }
  for (int64_t a0 = 0; a0 < m; a0 += kCylStep) {
    double pv[kCylStep], l1[kCylStep], l2[kCylStep], nb[kCylRhs][kCylStep];
#pragma unroll
    for (int t = 0; t < kCylStep; ++t) {
      const int64_t a = a0 + t;
      const double *f = f0 + (a < m ? a : 0) * npad;
      pv[t] = f[0];
      l1[t] = f[fs];
      l2[t] = f[2 * fs];
#pragma unroll
      for (int r = 0; r < kCylRhs; ++r) nb[r][t] = a + 3 < m ? b[r][(a + 3) * npad] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kCylStep; ++t) {
      const int64_t a = a0 + t;
      if (a >= m) break;
      const int p = (int)pv[t];
#pragma unroll
      for (int r = 0; r < kCylRhs; ++r) {
        if (p == 1) {
          const double tt = w0[r];
          w0[r] = w1[r];
          w1[r] = tt;
        } else if (p == 2) {
          const double tt = w0[r];
          w0[r] = w2[r];
          w2[r] = tt;
        }
        w1[r] -= l1[t] * w0[r];
        w2[r] -= l2[t] * w0[r];
        if (use[r]) b[r][a * npad] = w0[r];
        w0[r] = w1[r];
        w1[r] = w2[r];
        w2[r] = nb[r][t];
      }
    }
  }
  double x1[kCylRhs], x2[kCylRhs], x3[kCylRhs], x4[kCylRhs];
#pragma unroll
  for (int r = 0; r < kCylRhs; ++r) x1[r] = x2[r] = x3[r] = x4[r] = 0.0;
  for (int64_t a1 = m - 1; a1 >= 0; a1 -= kCylStep) {
    double iu[kCylStep], u1[kCylStep], u2[kCylStep], u3[kCylStep], u4[kCylStep];
    double bv[kCylRhs][kCylStep];
#pragma unroll
    for (int t = 0; t < kCylStep; ++t) {
      const int64_t a = a1 - t >= 0 ? a1 - t : 0;
      const double *f = f0 + a * npad;
      iu[t] = f[3 * fs];
      u1[t] = f[4 * fs];
      u2[t] = f[5 * fs];
      u3[t] = f[6 * fs];
      u4[t] = f[7 * fs];
#pragma unroll
      for (int r = 0; r < kCylRhs; ++r) bv[r][t] = b[r][a * npad];
    }
#pragma unroll
    for (int t = 0; t < kCylStep; ++t) {
      const int64_t a = a1 - t;
      if (a < 0) break;
#pragma unroll
      for (int r = 0; r < kCylRhs; ++r) {
        const double v =
            (bv[r][t] - u1[t] * x1[r] - u2[t] * x2[r] - u3[t] * x3[r] - u4[t] * x4[r]) * iu[t];
        if (use[r]) x[r][a * npad] = v;
        x4[r] = x3[r];
        x3[r] = x2[r];
        x2[r] = x1[r];
        x1[r] = v;
      }
    }
  }
  for (int64_t a = m; a < mp; ++a)
#pragma unroll
    for (int r = 0; r < kCylRhs; ++r)
      if (use[r]) x[r][a * npad] = 0.0;
}

// Thin edges of the r output map (see launch_cyl_redge).  The edge
// columns of X0_blk and the edge rows of Pr are staged in LDS.  Tasks: the rows i < ro_main of the
// column edge (reading PrT coalesced, threads over rows) and the columns
// j < mo of the row edge (reading X0_blk coalesced, threads over columns),
// one task per thread; the
// k loops load kCylEdgeB values before using them.
constexpr int kCylEdgeMax = 8, kCylEdgeK = 256, kCylEdgeB = 16, kCylEdgeThreads = 320;

__global__ __launch_bounds__(kCylEdgeThreads) void k_cyl_redge(
    const CylEdge *__restrict__ d, char *ws, double *__restrict__ U, int64_t mp, int64_t ro,
    int64_t ro_main, int64_t mo, int64_t mo_main, int64_t mobar, int64_t ldc) {
  __shared__ double xs[kCylEdgeMax][kCylEdgeK];  // X0_blk columns mo_main..
  __shared__ double ps[kCylEdgeMax][kCylEdgeK];  // Pr rows ro_main..
  const CylEdge &e = d[blockIdx.x];
  const double *__restrict__ B = (const double *)(ws + e.b_off);
  double *__restrict__ C = U + e.c_off;
  const int ne_c = (int)(mo - mo_main), ne_r = (int)(ro - ro_main);
  const int tid = threadIdx.x;
  for (int64_t t = tid; t < ne_c * mp; t += kCylEdgeThreads) {
    const int64_t c = t / mp, k = t % mp;
    xs[c][k] = B[k * mobar + mo_main + c];
  }
  for (int64_t t = tid; t < ne_r * mp; t += kCylEdgeThreads) {
    const int64_t r = t / mp, k = t % mp;
    ps[r][k] = e.Pr[(ro_main + r) * mp + k];
  }
  __syncthreads();
  const int64_t ntask = (ne_c > 0 ? ro_main : 0) + (ne_r > 0 ? mo : 0);
  for (int64_t task = tid; task < ntask; task += kCylEdgeThreads) {
    double acc[kCylEdgeMax];
#pragma unroll
    for (int r = 0; r < kCylEdgeMax; ++r) acc[r] = 0.0;
    if (ne_c > 0 && task < ro_main) {  // column edge, row i
      const int64_t i = task;
      for (int64_t k0 = 0; k0 < mp; k0 += kCylEdgeB) {
        double a[kCylEdgeB];
#pragma unroll
        for (int u = 0; u < kCylEdgeB; ++u) a[u] = e.PrT[(k0 + u) * ro + i];
#pragma unroll
        for (int u = 0; u < kCylEdgeB; ++u)
#pragma unroll
          for (int c = 0; c < kCylEdgeMax; ++c)
            if (c < ne_c) acc[c] = fma(a[u], xs[c][k0 + u], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < kCylEdgeMax; ++c)
        if (c < ne_c) C[i * ldc + (mo_main + c) * 2] = acc[c];
    } else {  // row edge, column j
      const int64_t j = task - (ne_c > 0 ? ro_main : 0);
      for (int64_t k0 = 0; k0 < mp; k0 += kCylEdgeB) {
        double b[kCylEdgeB];
#pragma unroll
        for (int u = 0; u < kCylEdgeB; ++u) b[u] = B[(k0 + u) * mobar + j];
#pragma unroll
        for (int u = 0; u < kCylEdgeB; ++u)
#pragma unroll
          for (int r = 0; r < kCylEdgeMax; ++r)
            if (r < ne_r) acc[r] = fma(ps[r][k0 + u], b[u], acc[r]);
      }
#pragma unroll
      for (int r = 0; r < kCylEdgeMax; ++r)
        if (r < ne_r) C[(ro_main + r) * ldc + j * 2] = acc[r];
    }
  }
}

}  // namespace

hipError_t launch_cyl_permute_in(const double *F, double *X0, const int *slot_idx, int64_t n,
                                 int64_t nt, int64_t mp, hipStream_t st) {
  const int64_t total = nt * 2 * (2 * mp) * mp;
  if (total <= 0) return hipSuccess;
  if (total >= ((int64_t)1 << 32) - 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cyl_permute_in, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, F,
                     X0, slot_idx, (uint32_t)n, (uint32_t)mp, (uint32_t)total);
  return hipGetLastError();
}

hipError_t launch_cyl_solve(double *X0, double *X1, const double *fac, const CylSolveGroup *grp,
                            int ngroups, int64_t m, int64_t mp, hipStream_t st) {
  const int64_t npad = 2 * mp;
  if (ngroups <= 0) return hipSuccess;
  dim3 grid((unsigned)((npad + 63) / 64), (unsigned)ngroups);
  hipLaunchKernelGGL(k_cyl_solve, grid, dim3(64), 0, st, X0, X1, fac, grp, m, mp);
  return hipGetLastError();
}

hipError_t launch_cyl_redge(const CylEdge *d, int nprob, char *ws, double *U, int64_t mp,
                            int64_t ro, int64_t ro_main, int64_t mo, int64_t mo_main,
                            int64_t mobar, int64_t ldc, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  if (mp > kCylEdgeK || mp % kCylEdgeB != 0 || mo - mo_main > kCylEdgeMax ||
      ro - ro_main > kCylEdgeMax || mo_main > mo || ro_main > ro)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cyl_redge, dim3((unsigned)nprob), dim3(kCylEdgeThreads), 0, st, d, ws, U, mp,
                     ro, ro_main, mo, mo_main, mobar, ldc);
  return hipGetLastError();
}

}  // namespace fps
