// gfx950 kernels of the cylinder solve: the input permutation into the
// parity-blocked per-mode layout and the banded solves in r (one thread per
// mode, real/imaginary part and z column, applying LU factors computed by
// the plan with partial pivoting).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

__device__ inline int64_t natural_of(int64_t pos, int64_t m, int64_t mp) {
  // parity-blocked position -> natural index, or -1 for padding
  const int s = pos >= mp ? 1 : 0;
  const int64_t a = pos - (s ? mp : 0);
  return a < m ? 2 * a + s : -1;
}

// X0[((slot * 2 + part) * npad + rpos) * npad + zpos] = F[idx][part][i][j]
// (zero at padded positions); grid (npad / 64, npad, nt * 2).
__global__ __launch_bounds__(64) void k_cyl_permute_in(const double *__restrict__ F,
                                                       double *__restrict__ X0,
                                                       const int *__restrict__ slot_idx,
                                                       int64_t n, int64_t mp) {
  const int64_t npad = 2 * mp, m = n / 2;
  const int64_t zpos = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t rpos = blockIdx.y;
  const int64_t sp = blockIdx.z;  // slot * 2 + part
  if (zpos >= npad) return;
  const int64_t i = natural_of(rpos, m, mp), j = natural_of(zpos, m, mp);
  const int64_t idx = slot_idx[sp >> 1], part = sp & 1;
  double v = 0.0;
  if (i >= 0 && j >= 0) v = F[((idx * 2 + part) * n + i) * n + j];
  X0[(sp * npad + rpos) * npad + zpos] = v;
}

// One banded system (Q_k + lambda_j P_k) yhat = rhs per thread.  rhs: X0 rows
// of parity rp (column zpos, stride npad), overwritten by the forward
// substitution; yhat: X1 rows of parity wp (zeros beyond m and for padded
// columns).  Factors fac[((kabs * 8 + t) * mp + a) * npad + zpos], t: pivot
// offset, two multipliers, 1/u_aa, four superdiagonal entries of U.
__global__ __launch_bounds__(64) void k_cyl_solve(double *__restrict__ X0,
                                                  double *__restrict__ X1,
                                                  const double *__restrict__ fac,
                                                  const int *__restrict__ slot_kabs,
                                                  const int *__restrict__ slot_rp,
                                                  const int *__restrict__ slot_wp, int64_t m,
                                                  int64_t mp) {
  const int64_t npad = 2 * mp;
  const int64_t zpos = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t sp = blockIdx.y;
  if (zpos >= npad) return;
  const int64_t slot = sp >> 1;
  const int64_t kabs = slot_kabs[slot], rp = slot_rp[slot], wp = slot_wp[slot];
  double *b = X0 + (sp * npad + rp * mp) * npad + zpos;
  double *x = X1 + (sp * npad + wp * mp) * npad + zpos;
  const int s = zpos >= mp ? 1 : 0;
  const bool valid = zpos - (s ? mp : 0) < m;
  if (!valid) {
    for (int64_t a = 0; a < mp; ++a) x[a * npad] = 0.0;
    return;
  }
  const double *f0 = fac + ((kabs * 8 + 0) * mp) * npad + zpos;
  const int64_t fs = mp * npad;  // between factor fields
  double w0 = b[0], w1 = m > 1 ? b[npad] : 0.0, w2 = m > 2 ? b[2 * npad] : 0.0;
  for (int64_t a = 0; a < m; ++a) {
    const double *f = f0 + a * npad;
    const int p = (int)f[0];
    if (p == 1) {
      const double t = w0;
      w0 = w1;
      w1 = t;
    } else if (p == 2) {
      const double t = w0;
      w0 = w2;
      w2 = t;
    }
    w1 -= f[fs] * w0;
    w2 -= f[2 * fs] * w0;
    b[a * npad] = w0;
    w0 = w1;
    w1 = w2;
    w2 = a + 3 < m ? b[(a + 3) * npad] : 0.0;
  }
  double x1 = 0.0, x2 = 0.0, x3 = 0.0, x4 = 0.0;
  for (int64_t a = m - 1; a >= 0; --a) {
    const double *f = f0 + a * npad;
    const double v = (b[a * npad] - f[4 * fs] * x1 - f[5 * fs] * x2 - f[6 * fs] * x3 -
                      f[7 * fs] * x4) * f[3 * fs];
    x[a * npad] = v;
    x4 = x3;
    x3 = x2;
    x2 = x1;
    x1 = v;
  }
  for (int64_t a = m; a < mp; ++a) x[a * npad] = 0.0;
}

}  // namespace

hipError_t launch_cyl_permute_in(const double *F, double *X0, const int *slot_idx, int64_t n,
                                 int64_t nt, int64_t mp, hipStream_t st) {
  const int64_t npad = 2 * mp;
  dim3 grid((unsigned)((npad + 63) / 64), (unsigned)npad, (unsigned)(nt * 2));
  hipLaunchKernelGGL(k_cyl_permute_in, grid, dim3(64), 0, st, F, X0, slot_idx, n, mp);
  return hipGetLastError();
}

hipError_t launch_cyl_solve(double *X0, double *X1, const double *fac, const int *slot_kabs,
                            const int *slot_rp, const int *slot_wp, int64_t m, int64_t mp,
                            int64_t nt, hipStream_t st) {
  const int64_t npad = 2 * mp;
  dim3 grid((unsigned)((npad + 63) / 64), (unsigned)(nt * 2));
  hipLaunchKernelGGL(k_cyl_solve, grid, dim3(64), 0, st, X0, X1, fac, slot_kabs, slot_rp, slot_wp,
                     m, mp);
  return hipGetLastError();
}

}  // namespace fps
