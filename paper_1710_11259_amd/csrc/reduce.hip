// gfx950 chunk-carry kernels of the ADI half-sweeps.  A sweep solves every
// chunk of every chain with zero carry-in and leaves two boundary values per
// chain and chunk; these kernels run the chunk-level recurrences of each
// chain (the shifted tridiagonal solves of Algorithm 2, one chain per parity
// block, partitioned into chunks) and write the carries that the next sweep
// folds into its input.
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
// Both recurrences are affine in the carry, so each is a prefix composition
// of affine maps z -> a z + b.  A chain gets a segment of kL lanes; lane l
// owns the q = ceil(nc / 16) consecutive chunks [l q, l q + q) and composes
// their maps serially, a Hillis-Steele scan over the segment (log2 kL
// shuffle steps each way) gives every lane the carry at its first chunk,
// and the lane expands its chunks serially from there.  Lanes without
// chunks hold the identity, so a chunk's result does not depend on kL.
// (A few chunks per lane keep the scan short: 4 shuffle steps at most,
// and a quarter of the wavefronts of one lane per chunk.)  A lane keeps its
// chunks' data and forward carries in registers (at most 8 chunks per lane:
// chains of up to 128 chunks).
// Lanes that a chain's scan spans at most, and the chunks each lane owns:
// a function of the chain's own chunk count only, so batched launches (whose
// segment width kL covers their longest chain) compute every chain exactly
// as its single launch does.
constexpr int kScanLanes = kReduceMaxLanes;
__device__ __forceinline__ int chunks_per_lane(int nc) {
  return (nc + kScanLanes - 1) / kScanLanes;
}

// Where one chain's chunk data sits: boundary values y (last forward value)
// and x (first backward value) of chunk k at k * ystride, coefficient slot
// j of chunk k at ct[j * ctstride + k]; global memory or the LDS stage.
struct ChainSrc {
  const double *y, *x;
  int64_t ystride;
  const double *ct;
  int64_t ctstride;
};

// The scan with at most kQ chunks per lane held in registers: every load is
// issued before the first use (one round of memory latency) and cf stays in
// registers.  o: the chain's output, chunk k at k * ostride (cf, cb).
template <int kL, int kQ>
__device__ __forceinline__ void reduce_chain_scan_reg(const ChainSrc &src, double *__restrict__ o,
                                                      int64_t ostride, double scale, int nc,
                                                      int lane) {
  const int q = chunks_per_lane(nc);  // <= kQ
  const int lo = lane * q < nc ? lane * q : nc;
  const int hi = lo + q < nc ? lo + q : nc;
  const double *__restrict__ ct = src.ct;
  const int64_t cs = src.ctstride, ys = src.ystride;
  double a[kQ], y[kQ], xn[kQ], bfn[kQ], bkn[kQ];
#pragma unroll
  for (int t = 0; t < kQ; ++t) {
    const int k = lo + t;
    const bool in = k < hi, nx = in && k + 1 < nc;
    a[t] = in ? ct[C_F2LAST * cs + k] : 1.0;
    y[t] = in ? src.y[(int64_t)k * ys] : 0.0;
    xn[t] = nx ? src.x[(int64_t)(k + 1) * ys] : 0.0;
    bfn[t] = nx ? ct[C_BF2FIRST * cs + k + 1] : 0.0;
    bkn[t] = nx ? ct[C_BK2FIRST * cs + k + 1] : 1.0;
  }
  double fa = 1.0, fb = 0.0;
#pragma unroll
  for (int t = 0; t < kQ; ++t)
    if (lo + t < hi) {
      fb = a[t] * fb + y[t];
      fa = a[t] * fa;
    }
#pragma unroll
  for (int d = 1; d < kL; d <<= 1) {
    const double pa = __shfl_up(fa, d, kL), pb = __shfl_up(fb, d, kL);
    if (lane >= d) {
      fb = fa * pb + fb;
      fa = fa * pa;
    }
  }
  double cf = __shfl_up(fb, 1, kL);
  if (lane == 0) cf = 0.0;
  double cfv[kQ];
  double ba = 1.0, bb = 0.0;
#pragma unroll
  for (int t = 0; t < kQ; ++t) {
    const int k = lo + t;
    cfv[t] = cf;
    if (k < hi) {
      cf = k + 1 == hi ? fb : a[t] * cf + y[t];
      if (k + 1 < nc) {
        const double c = xn[t] + bfn[t] * cf;
        bb = ba * c + bb;
        ba = ba * bkn[t];
      }
    }
  }
#pragma unroll
  for (int d = 1; d < kL; d <<= 1) {
    const double na = __shfl_down(ba, d, kL), nb = __shfl_down(bb, d, kL);
    if (lane + d < kL) {
      bb = ba * nb + bb;
      ba = ba * na;
    }
  }
  double cb = __shfl_down(bb, 1, kL);
  if (lane + 1 >= kL) cb = 0.0;
  double cfn = fb;
#pragma unroll
  for (int t = kQ - 1; t >= 0; --t) {
    const int k = lo + t;
    if (k < hi) {
      const double cfk = cfv[t];
      if (k == lo)
        cb = bb;
      else if (k + 1 < nc)
        cb = bkn[t] * cb + (xn[t] + bfn[t] * cfn);
      else
        cb = 0.0;
      o[(int64_t)k * ostride] = scale * cfk;
      o[(int64_t)k * ostride + 1] = scale * cb;
      cfn = cfk;
    }
  }
}

// The carries of the workgroup's kReduceThreads / kL chains (r0 .., below
// rend) of parity s.
template <int kL, int kQ>
__device__ __forceinline__ void reduce_block(const double *__restrict__ lv,
                                             const double *__restrict__ ct,
                                             double *__restrict__ ab, double scale,
                                             int64_t nchains, int nc, int64_t ncmax, int s,
                                             int64_t r0, int64_t rend) {
  const int ch = threadIdx.x / kL, lane = threadIdx.x % kL;
  const int64_t r = r0 + ch;
  if (r >= rend || nc == 0) return;  // whole kL-lane segments leave together
  const double *yl = lv + (int64_t)s * 2 * nchains + r;
  const ChainSrc src{yl, yl + nchains, 4 * nchains, ct, ncmax};
  reduce_chain_scan_reg<kL, kQ>(src, ab + ((int64_t)s * ncmax * nchains + r) * 2, 2 * nchains,
                                scale, nc, lane);
}

// Grid: (ceil((r_hi - r_lo) / (kReduceThreads / kL)), parities s_lo ..,
// batch); workgroup of kReduceThreads threads, chain-major.
template <int kL, int kQ>
__global__ __launch_bounds__(kReduceThreads) void k_reduce(
    const double *__restrict__ lv, const double *__restrict__ ctab, double *__restrict__ ab,
    double scale, int64_t nchains, int nc0, int nc1, int64_t ncmax, int64_t lvb, int64_t abb,
    int64_t r_lo, int64_t r_hi, int s_lo) {
  const int s = (int)blockIdx.y + s_lo;
  const int nc = s ? nc1 : nc0;
  const int64_t z = blockIdx.z;
  reduce_block<kL, kQ>(lv + z * lvb, ctab + (int64_t)s * kNCTab * ncmax, ab + z * abb, scale,
                       nchains, nc, ncmax, s,
                       r_lo + (int64_t)blockIdx.x * (kReduceThreads / kL), r_hi);
}

template <int kL, int kQ>
__global__ __launch_bounds__(kReduceThreads) void k_reduce_batch(
    const BatchReduce *__restrict__ d, const int *__restrict__ wg_prob, char *base, int wg_base) {
  const int g = (int)blockIdx.x + wg_base;
  const int k = __builtin_amdgcn_readfirstlane(wg_prob[g]);
  const BatchReduce &e = d[k];
  const int local = g - e.wg_start;
  const int s = local / e.nbx;
  const int nc = s ? e.nc1 : e.nc0;
  reduce_block<kL, kQ>((const double *)(base + e.lv_off), e.ctab + (int64_t)s * kNCTab * e.ncmax,
                       (double *)(base + e.ab_off), e.scale, e.npad, nc, e.ncmax, s,
                       (int64_t)(local % e.nbx) * (kReduceThreads / kL), e.npad);
}

// Kernel shape for chains of up to ncmax chunks: lanes per chain, and the
// bound kQ of chunks per lane held in registers (0: more than 8 chunks per
// lane, i.e. more than 128 per chain, which no plan creates).
void reduce_shape(int64_t ncmax, int *lanes, int *kq) {
  *lanes = reduce_lanes(ncmax);
  const int64_t q = (ncmax + kScanLanes - 1) / kScanLanes;
  *kq = q <= 1 ? 1 : q <= 2 ? 2 : q <= 4 ? 4 : q <= 8 ? 8 : 0;
}

}  // namespace

// Expands LAUNCH(L, Q) for the instantiated shape (lanes, kq).
#define FPS_WITH_REDUCE_SHAPE(lanes, kq, LAUNCH) \
  do {                                           \
    if ((lanes) == 2)                            \
      LAUNCH(2, 1);                              \
    else if ((lanes) == 4)                       \
      LAUNCH(4, 1);                              \
    else if ((lanes) == 8)                       \
      LAUNCH(8, 1);                              \
    else if ((kq) == 1)                          \
      LAUNCH(16, 1);                             \
    else if ((kq) == 2)                          \
      LAUNCH(16, 2);                             \
    else if ((kq) == 4)                          \
      LAUNCH(16, 4);                             \
    else if ((kq) == 8)                          \
      LAUNCH(16, 8);                             \
    else                                         \
      return hipErrorInvalidValue;               \
  } while (0)

hipError_t launch_reduce(const double *lv, const double *ctab, double *ab, double scale,
                         int64_t nchains, int nc0, int nc1, int64_t ncmax, hipStream_t st,
                         int nbatch, int64_t lvb, int64_t abb, int64_t r_lo, int64_t r_hi,
                         int s_lo, int s_hi) {
  if (r_hi < 0) r_hi = nchains;
  if (r_lo < 0 || r_hi > nchains || s_lo < 0 || s_hi > 2) return hipErrorInvalidValue;
  if (r_lo >= r_hi || s_lo >= s_hi) return hipSuccess;
  const int chains = reduce_chains(ncmax);
  dim3 grid((unsigned)((r_hi - r_lo + chains - 1) / chains), (unsigned)(s_hi - s_lo),
            (unsigned)(nbatch > 0 ? nbatch : 1));
  int lanes, kq;
  reduce_shape(ncmax, &lanes, &kq);
#define FPS_LAUNCH(L, Q)                                                                    \
  hipLaunchKernelGGL((k_reduce<L, Q>), grid, dim3(kReduceThreads), 0, st, lv, ctab, ab, \
                     scale, nchains, nc0, nc1, ncmax, lvb, abb, r_lo, r_hi, s_lo)
  FPS_WITH_REDUCE_SHAPE(lanes, kq, FPS_LAUNCH);
#undef FPS_LAUNCH
  return hipGetLastError();
}

hipError_t launch_reduce_batch(const BatchReduce *d, const int *wg_prob, int nwg, int64_t ncmax_max,
                               char *base, hipStream_t st, int wg_base) {
  if (nwg <= 0) return hipSuccess;
  int lanes, kq;
  reduce_shape(ncmax_max, &lanes, &kq);
#define FPS_LAUNCH(L, Q)                                                                     \
  hipLaunchKernelGGL((k_reduce_batch<L, Q>), dim3((unsigned)nwg), dim3(kReduceThreads), 0, \
                     st, d, wg_prob, base, wg_base)
  FPS_WITH_REDUCE_SHAPE(lanes, kq, FPS_LAUNCH);
#undef FPS_LAUNCH
  return hipGetLastError();
}

#undef FPS_WITH_REDUCE_SHAPE

}  // namespace fps
