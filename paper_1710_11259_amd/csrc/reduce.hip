// gfx950 chunk-carry kernels of the ADI half-sweeps.  A sweep solves every
// chunk of every chain with zero carry-in and leaves two boundary values per
// chain and chunk; these kernels run the chunk-level recurrences of each
// chain (App. D.4 systems, partitioned) and write the carries that the next
// sweep folds into its input.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

// Chunk carries of one half-sweep, per (parity s, chain r): the chunk-level
// recurrences on the chunk boundary values
//   cf[0] = 0,        cf[c+1] = ylast[c] + F2last[c] cf[c],
//   cb[nc-1] = 0,     cb[c] = xfirst[c+1] + BF2first[c+1] cf[c+1]
//                            + Bk2first[c+1] cb[c+1],
// (per-chunk coefficients ctab of the producing pass's shift), written as
// ab[s][c][r] = scale (cf[c], cb[c]).
//
// Sequential form (one thread per chain; used when a chain has more chunks
// than the lanes given to it).  cf is parked in ab between the two sweeps
// over the chunks (each thread rereads only what it wrote).
__device__ __forceinline__ void reduce_chain(const double *__restrict__ lv,
                                             const double *__restrict__ ct, double *__restrict__ ab,
                                             double scale, int64_t nchains, int nc, int64_t ncmax,
                                             int s, int64_t r) {
  const double *__restrict__ yl = lv + (int64_t)s * 2 * nchains + r;  // chunk q at q * 4 nchains
  const double *__restrict__ xf = yl + nchains;
  double *__restrict__ o = ab + ((int64_t)s * ncmax * nchains + r) * 2;  // chunk c at c * 2 nchains
  // forward: cf[c] parked (unscaled) in o[c][0]
  double cf = 0.0;
  for (int c0 = 0; c0 < nc; c0 += 8) {
    double y8[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) y8[k] = c0 + k < nc ? yl[(int64_t)(c0 + k) * 4 * nchains] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int c = c0 + k;
      if (c < nc) {
        o[(int64_t)c * 2 * nchains] = cf;
        cf = y8[k] + ct[C_F2LAST * ncmax + c] * cf;
      }
    }
  }
  // backward, chunks nc-1 .. 0; cfn = unscaled cf of chunk c + 1
  double cb = 0.0, cfn = 0.0;
  for (int c1 = nc - 1; c1 >= 0; c1 -= 8) {
    double f8[8], x8[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int c = c1 - k;
      f8[k] = c >= 0 ? o[(int64_t)c * 2 * nchains] : 0.0;
      x8[k] = c >= 0 && c + 1 < nc ? xf[(int64_t)(c + 1) * 4 * nchains] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int c = c1 - k;
      if (c >= 0) {
        cb = c + 1 < nc ? x8[k] + ct[C_BF2FIRST * ncmax + c + 1] * cfn +
                              ct[C_BK2FIRST * ncmax + c + 1] * cb
                        : 0.0;
        double *oc = o + (int64_t)c * 2 * nchains;
        oc[0] = scale * f8[k];
        oc[1] = scale * cb;
        cfn = f8[k];
      }
    }
  }
}

// Both recurrences are affine in the carry, so each is a prefix composition
// of affine maps z -> a z + b: lane c of the chain's kL-lane segment holds
// chunk c's map, and a Hillis-Steele scan over the segment (log2 kL
// shuffle steps each way) gives every chunk its carry with one round of
// loads and one of stores.  Lanes at and beyond nc hold the identity, so
// the result of a chunk does not depend on kL.
template <int kL>
__device__ __forceinline__ void reduce_chain_scan(const double *__restrict__ lv,
                                                  const double *__restrict__ ct,
                                                  double *__restrict__ ab, double scale,
                                                  int64_t nchains, int nc, int64_t ncmax, int s,
                                                  int64_t r, int c) {
  const double *__restrict__ yl = lv + (int64_t)s * 2 * nchains + r;  // chunk q at q * 4 nchains
  const double *__restrict__ xf = yl + nchains;
  double fa = 1.0, fb = 0.0;  // cf[c+1] = fa cf[c] + fb
  double xn = 0.0, bf = 0.0, bk = 1.0;
  if (c < nc) {
    fa = ct[C_F2LAST * ncmax + c];
    fb = yl[(int64_t)c * 4 * nchains];
  }
  const bool inner = c + 1 < nc;
  if (inner) {
    xn = xf[(int64_t)(c + 1) * 4 * nchains];
    bf = ct[C_BF2FIRST * ncmax + c + 1];
    bk = ct[C_BK2FIRST * ncmax + c + 1];
  }
#pragma unroll
  for (int d = 1; d < kL; d <<= 1) {  // fb <- cf[c+1]
    const double pa = __shfl_up(fa, d, kL), pb = __shfl_up(fb, d, kL);
    if (c >= d) {
      fb = fa * pb + fb;
      fa = fa * pa;
    }
  }
  double cf = __shfl_up(fb, 1, kL);
  if (c == 0) cf = 0.0;
  // cb[c] = ba cb[c+1] + bb; the last chunk's map is the identity (cb = 0)
  double ba = bk, bb = inner ? xn + bf * fb : 0.0;
#pragma unroll
  for (int d = 1; d < kL; d <<= 1) {  // bb <- cb[c]
    const double na = __shfl_down(ba, d, kL), nb = __shfl_down(bb, d, kL);
    if (c + d < kL) {
      bb = ba * nb + bb;
      ba = ba * na;
    }
  }
  if (c < nc) {
    double *oc = ab + (((int64_t)s * ncmax + c) * nchains + r) * 2;
    oc[0] = scale * cf;
    oc[1] = scale * bb;
  }
}

// One chain on kL lanes: the scan when its chunks fit, else lane 0 runs the
// sequential form.
template <int kL>
__device__ __forceinline__ void reduce_one(const double *lv, const double *ct, double *ab,
                                           double scale, int64_t nchains, int nc, int64_t ncmax,
                                           int s, int64_t r, int c) {
  if (nc <= kL)
    reduce_chain_scan<kL>(lv, ct, ab, scale, nchains, nc, ncmax, s, r, c);
  else if (c == 0)
    reduce_chain(lv, ct, ab, scale, nchains, nc, ncmax, s, r);
}

// Grid: (ceil(nchains / kReduceChains), 2 parities, batch); workgroup of
// kReduceChains x kL threads, chain-major.
template <int kL>
__global__ __launch_bounds__(kReduceChains * kL) void k_reduce(
    const double *__restrict__ lv, const double *__restrict__ ctab, double *__restrict__ ab,
    double scale, int64_t nchains, int nc0, int nc1, int64_t ncmax, int64_t lvb, int64_t abb) {
  const int s = blockIdx.y;
  const int nc = s ? nc1 : nc0;
  const int64_t r = (int64_t)blockIdx.x * kReduceChains + threadIdx.x / kL;
  if (r >= nchains || nc == 0) return;  // whole kL-lane segments leave together
  const int64_t z = blockIdx.z;
  reduce_one<kL>(lv + z * lvb, ctab + (int64_t)s * kNCTab * ncmax, ab + z * abb, scale, nchains,
                 nc, ncmax, s, r, (int)(threadIdx.x % kL));
}

template <int kL>
__global__ __launch_bounds__(kReduceChains * kL) void k_reduce_batch(
    const BatchReduce *__restrict__ d, const int *__restrict__ wg_prob, char *base) {
  const int k = __builtin_amdgcn_readfirstlane(wg_prob[blockIdx.x]);
  const BatchReduce &e = d[k];
  const int local = (int)blockIdx.x - e.wg_start;
  const int s = local / e.nbx;
  const int nc = s ? e.nc1 : e.nc0;
  const int64_t r = (int64_t)(local % e.nbx) * kReduceChains + threadIdx.x / kL;
  if (r >= e.npad || nc == 0) return;
  reduce_one<kL>((const double *)(base + e.lv_off), e.ctab + (int64_t)s * kNCTab * e.ncmax,
                 (double *)(base + e.ab_off), e.scale, e.npad, nc, e.ncmax, s, r,
                 (int)(threadIdx.x % kL));
}

// Lanes per chain: the least power of two from 2 to 64 that holds ncmax
// chunks (64 beyond; chains longer than that take the sequential form).
int reduce_lanes(int64_t ncmax) {
  int l = 2;
  while (l < 64 && l < ncmax) l <<= 1;
  return l;
}

}  // namespace

hipError_t launch_reduce(const double *lv, const double *ctab, double *ab, double scale,
                         int64_t nchains, int nc0, int nc1, int64_t ncmax, hipStream_t st,
                         int nbatch, int64_t lvb, int64_t abb) {
  dim3 grid((unsigned)((nchains + kReduceChains - 1) / kReduceChains), 2u,
            (unsigned)(nbatch > 0 ? nbatch : 1));
  const int lanes = reduce_lanes(ncmax);
#define FPS_REDUCE(L)                                                                        \
  hipLaunchKernelGGL(k_reduce<L>, grid, dim3(kReduceChains * L), 0, st, lv, ctab, ab, scale, \
                     nchains, nc0, nc1, ncmax, lvb, abb)
  if (lanes == 2)
    FPS_REDUCE(2);
  else if (lanes == 4)
    FPS_REDUCE(4);
  else if (lanes == 8)
    FPS_REDUCE(8);
  else if (lanes == 16)
    FPS_REDUCE(16);
  else if (lanes == 32)
    FPS_REDUCE(32);
  else
    FPS_REDUCE(64);
#undef FPS_REDUCE
  return hipGetLastError();
}

hipError_t launch_reduce_batch(const BatchReduce *d, const int *wg_prob, int nwg, int64_t ncmax_max,
                               char *base, hipStream_t st) {
  if (nwg <= 0) return hipSuccess;
  const int lanes = reduce_lanes(ncmax_max);
#define FPS_REDUCE(L)                                                                      \
  hipLaunchKernelGGL(k_reduce_batch<L>, dim3((unsigned)nwg), dim3(kReduceChains * L), 0, st, d, \
                     wg_prob, base)
  if (lanes == 2)
    FPS_REDUCE(2);
  else if (lanes == 4)
    FPS_REDUCE(4);
  else if (lanes == 8)
    FPS_REDUCE(8);
  else if (lanes == 16)
    FPS_REDUCE(16);
  else if (lanes == 32)
    FPS_REDUCE(32);
  else
    FPS_REDUCE(64);
#undef FPS_REDUCE
  return hipGetLastError();
}

}  // namespace fps
