// gfx950 row-chain ADI half-sweep: the shifted tridiagonal solves of
// Algorithm 2 along the storage rows of an array (one chain per row and
// parity block of its columns), with its output stored in place of its
// input's layout.  With this pass solving along rows and the column-chain
// sweep (sweep.hip) along columns, neither half-step has to transpose: both
// read and write their tiles row by row.
//
// Arithmetic is that of the column-chain sweep, position by position (the
// same whole-chain Thomas factors, the same segment-carry combinations in
// the same order, the same chunk boundary values), so a row-chain pass on an
// array equals a column-chain pass on its transpose bit for bit.  Only the
// distribution differs: the workgroup's 32 x 64 tile is loaded and stored
// with one column per lane (every instruction moves one 64-position run of
// a row, as in the column-chain pass) and turned around in LDS, so that a
// wavefront holds 8 chains, each split over 8 consecutive lanes of kSeg
// positions; the carries between the segments of a chunk are exchanged
// through the wavefront's own LDS row.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

constexpr int kRWaves = 4;                 // wavefronts per workgroup
constexpr int kRThreads = 64 * kRWaves;    // 256: 32 chains x 8 segments
constexpr int kRSegs = kChunk / kSeg;      // segments per chunk (8)
constexpr int kChainsPerWave = 64 / kRSegs;
static_assert(kRSegs == kWaves, "segment-carry combinations are indexed by segment");
constexpr int kRChains = kChainsPerWave * kRWaves;  // chains (rows) per workgroup
static_assert(kChunk % kRChains == 0, "a workgroup's rows lie in one chunk of the producer");
static_assert(kSeg * kRWaves == kRChains, "the column-wise phases cover the tile's rows");

// LDS (doubles): the chunk's per-position tables and segment-carry
// combinations, one exchange row per wavefront, and the tile.
constexpr int RO_TAB = 0;
constexpr int RO_L1 = RO_TAB + 5 * kChunk;
// Per wavefront and lane: the segment end values (forward, then backward),
// then the segment's backward-carry coefficient.
constexpr int RO_X = RO_L1 + kL1;
// The 32 x 64 tile (rows = chains, columns = positions; row stride kTS keeps
// every lane's segment 16-byte aligned): loaded and stored row by row with
// one column per lane, read and written segment by segment with one chain
// segment per lane.
constexpr int kTS = kChunk + 2;
constexpr int RO_T = RO_X + kRWaves * 64;
constexpr int RO_END = RO_T + kRChains * kTS;
static_assert(RO_T % 2 == 0 && kTS % 2 == 0 && kSeg % 2 == 0, "16-byte aligned segments");
static_assert(T_L == 0 && T_IB == 1 && T_U == 2 && T_F1 == 3 && T_BK1 == 4, "table slot order");

typedef double dbl2 __attribute__((ext_vector_type(2)));

// Component k of the producer's chunk carry of its chain r at its chunk cp
// (parity sp), formed from its boundary values for chains of at most two
// chunks (as the column-chain sweep forms it).
__device__ __forceinline__ double fused_carry_rows(const SweepArgs &a, int sp, int64_t cp,
                                                   int64_t r, int k) {
  const int ncs = sp ? a.nc1 : a.nc0;
  if (ncs < 2 || (cp == 0) == (k == 0)) return 0.0;
  const int64_t nch = a.npad;
  const double y0 = a.lv_prev[((int64_t)(0 * 2 + sp) * 2 + 0) * nch + r];
  if (k == 0) return a.carry_scale * y0;
  const double x1 = a.lv_prev[((int64_t)(1 * 2 + sp) * 2 + 1) * nch + r];
  const double bf = a.ctab_prev[((int64_t)sp * kNCTab + C_BF2FIRST) * a.ncmax + 1];
  return a.carry_scale * (x1 + bf * y0);
}

// One workgroup: chunk `by` = blockIdx.x of the columns (parity-0 chunks
// first) of the chains (rows) bx * 32 .. bx * 32 + 31, bx = blockIdx.y.  Per
// lane in the row phase: chain bx * 32 + w * 8 + lane / 8, segment lane % 8
// (kSeg columns); in the load and store phases: column lane, rows w * 8 ..
// w * 8 + 7.  Four wavefronts per workgroup keep the register- and
// LDS-bound occupancy in whole workgroups.
//   v   = in_scale * in + (chunk carries of the producing pass)
//   x   = T^-1 v with T the pass's tridiagonal (tables)
//   out = x (out_mode 1) or v - sigma x (out_mode 2), stored like `in`.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kRThreads) void k_sweep_rows(SweepArgs a) {
  __shared__ double lds[RO_END];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int seg = lane % kRSegs;
  const int by = blockIdx.x;
  const int s = by < a.nc0 ? 0 : 1;
  const int c = by - (s ? a.nc0 : 0);
  const int64_t mps = s ? a.mp1 : a.mp0;
  const int64_t kc0 = (int64_t)c * kChunk;
  const int64_t cbase = (s ? a.mp0 : 0) + kc0;  // first column of the chunk
  const int64_t rblk = (int64_t)blockIdx.y * kRChains;
  const int64_t row = rblk + w * kChainsPerWave + lane / kRSegs;
  const int64_t ld = a.ld, ms = a.mstride, ncmax = a.ncmax, npad = a.npad;
  const bool has_prev = a.tab_prev != nullptr;

  // Small values: this chunk's tables and combinations.
  const double *__restrict__ tab = a.tab + (int64_t)s * kNTab * ms + kc0;
  double tv = 0.0, tv2 = 0.0, l1v;
  if (tid < 5 * kChunk) tv = tab[(tid / kChunk) * ms + (tid % kChunk)];
  if (tid + kRThreads < 5 * kChunk)
    tv2 = tab[((tid + kRThreads) / kChunk) * ms + ((tid + kRThreads) % kChunk)];
  l1v = a.l1[((int64_t)s * ncmax + c) * kL1 + (tid < kL1 ? tid : kL1 - 1)];
  // The tile, one column per lane and kSeg rows per wavefront (every load
  // instruction reads one 64-position run of a row), with the producer's
  // carries folded in: its chains are this chunk's columns, its positions
  // this workgroup's rows (all in its chunk cp of parity sp), so the carry
  // of element (row, column) is ab[column] . (BF2, Bk2)[row].
  double y[kSeg];
  {
    const Tin *__restrict__ in = (const Tin *)a.in + (rblk + w * kSeg) * ld + cbase + lane;
#pragma unroll
    for (int i = 0; i < kSeg; ++i) y[i] = (double)in[i * ld];
  }
  {
    const double act = kc0 + (lane / kSeg) * kSeg < mps ? 1.0 : 0.0;  // segment of this column
    const double isc = act * a.in_scale;
    if (has_prev) {
      const int sp = rblk >= a.mp0 ? 1 : 0;
      const int64_t cp = (rblk - (sp ? a.mp0 : 0)) / kChunk;
      double acf, acb;
      if (a.ctab_prev != nullptr) {
        acf = fused_carry_rows(a, sp, cp, cbase + lane, 0);
        acb = fused_carry_rows(a, sp, cp, cbase + lane, 1);
      } else {
        const double *e = a.ab_prev + (((int64_t)sp * ncmax + cp) * npad + cbase + lane) * 2;
        acf = e[0];
        acb = e[1];
      }
      const double *tp = a.tab_prev + (int64_t)sp * kNTab * ms + (rblk + w * kSeg - (sp ? a.mp0 : 0));
#pragma unroll
      for (int i = 0; i < kSeg; ++i) {
        const double cA = act * tp[T_BF2 * ms + i], cB = act * tp[T_BK2 * ms + i];
        y[i] = isc * y[i] + acf * cA + acb * cB;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kSeg; ++i) y[i] = isc * y[i] + 0.0 * 0.0 + 0.0 * 0.0;
    }
  }
  if (tid < 5 * kChunk) lds[RO_TAB + tid] = tv;
  if (tid + kRThreads < 5 * kChunk) lds[RO_TAB + tid + kRThreads] = tv2;
  if (tid < kL1) lds[RO_L1 + tid] = l1v;
#pragma unroll
  for (int i = 0; i < kSeg; ++i) lds[RO_T + (w * kSeg + i) * kTS + lane] = y[i];
  __syncthreads();
  // this lane's chain segment
  double *Tseg = lds + RO_T + (w * kChainsPerWave + lane / kRSegs) * kTS + seg * kSeg;
#pragma unroll
  for (int i = 0; i < kSeg; i += 2) {
    const dbl2 t = *(const dbl2 *)(Tseg + i);
    y[i] = t.x;
    y[i + 1] = t.y;
  }
  const double *Tl = lds + RO_TAB + 0 * kChunk + seg * kSeg;
  const double *Tib = lds + RO_TAB + 1 * kChunk + seg * kSeg;
  const double *Tu = lds + RO_TAB + 2 * kChunk + seg * kSeg;
  const double *Tf1 = lds + RO_TAB + 3 * kChunk + seg * kSeg;
  const double *Tbk1 = lds + RO_TAB + 4 * kChunk + seg * kSeg;
  const double *L1f = lds + RO_L1 + (0 * kWaves + seg) * kWaves;
  const double *L1b = lds + RO_L1 + (1 * kWaves + seg) * kWaves;

  // Forward elimination with zero carry-in, then the segment carry from the
  // segments' last values (lanes of the same chain).  Scheduling barriers
  // between the phases keep each phase's table reads (LDS) from being
  // hoisted into the previous one, where all 40 per-lane table values would
  // be live at once.
  {
    double carry = 0.0;
#pragma unroll
    for (int i = 0; i < kSeg; ++i) {
      y[i] = y[i] - Tl[i] * carry;
      carry = y[i];
    }
  }
  // The 8 segment values of this lane's chain are adjacent in the wave's
  // LDS row (written and read by the same wavefront: no barrier).
  double *X = lds + RO_X + w * 64;
  const double *Xg = X + (lane & ~(kRSegs - 1));
  double cf1 = 0.0;
  X[lane] = y[kSeg - 1];
#pragma unroll
  for (int k = 0; k < kRSegs; ++k) cf1 += L1f[k] * Xg[k];
#pragma unroll
  for (int i = 0; i < kSeg; ++i) y[i] += Tf1[i] * cf1;
  const double ylast_chunk = y[kSeg - 1];
  __builtin_amdgcn_sched_barrier(0);

  // Chunk boundary value of the forward pass.
  const int64_t nch = a.ncols;
  if (seg == kRSegs - 1) a.lv[(((int64_t)c * 2 + s) * 2 + 0) * nch + row] = ylast_chunk;

  // Backward substitution with zero carry-in, fused with the output; the
  // right-hand side is recovered from the forward values.  The outputs go
  // back into the tile at once (each lane rewrites the positions it read).
  const double sigma = a.sigma;
  const bool out_x = a.out_mode == 1;
  double xnext = 0.0, xfirst = 0.0, onext = 0.0;
#pragma unroll
  for (int i = kSeg - 1; i >= 0; --i) {
    const double x = y[i] * Tib[i] - Tu[i] * xnext;
    const double rhs = y[i] + Tl[i] * (i > 0 ? y[i - 1] : cf1);
    const double o = out_x ? x : rhs - sigma * x;
    if (i % 2 == 0) *(dbl2 *)(Tseg + i) = dbl2{o, onext};
    onext = o;
    xnext = x;
    if (i == 0) xfirst = x;
  }
  __builtin_amdgcn_sched_barrier(0);
  double cb1 = 0.0;
  X[lane] = xfirst;
#pragma unroll
  for (int k = 0; k < kRSegs; ++k) cb1 += L1b[k] * Xg[k];
  // The backward carry enters every output of the segment as coef * Bk1;
  // it is added when the tile is stored (one coefficient per chain segment
  // in LDS, at the chain's row and the segment's index).
  const double coef = (out_x ? 1.0 : -sigma) * cb1;
  X[lane] = coef;  // after every lane of the wavefront has read its xfirst values
  if (seg == 0) a.lv[(((int64_t)c * 2 + s) * 2 + 1) * nch + row] = xfirst + Tbk1[0] * cb1;
  __syncthreads();
  // Stored row by row like the load: y + coef * Bk1 per position.
  Tout *__restrict__ out = (Tout *)a.out + (rblk + w * kSeg) * ld + cbase + lane;
  if (kc0 + lane < mps) {
    const double bk1 = lds[RO_TAB + 4 * kChunk + lane];
#pragma unroll
    for (int i = 0; i < kSeg; ++i) {
      const double yo = lds[RO_T + (w * kSeg + i) * kTS + lane];
      out[i * ld] = (Tout)(yo + lds[RO_X + w * 64 + i * kRSegs + lane / kSeg] * bk1);
    }
  }
}

}  // namespace

hipError_t launch_sweep_rows(const SweepArgs &a, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int nchunks = a.nc0 + a.nc1;
  if (a.npad % kChunk != 0 || a.ncols % kRChains != 0 || nchunks <= 0 || a.in == nullptr ||
      a.out == nullptr)
    return hipErrorInvalidValue;
  if (a.ncols != a.npad || a.ld < a.npad || a.ld % 4 != 0) return hipErrorInvalidValue;
  if (a.out_mode != 1 && a.out_mode != 2) return hipErrorInvalidValue;
  if (a.g != nullptr || a.pre != nullptr || a.nbatch > 1) return hipErrorInvalidValue;
  if (a.ctab_prev != nullptr) {
    if (a.tab_prev == nullptr || a.lv_prev == nullptr || a.ncmax > 2) return hipErrorInvalidValue;
  } else if ((a.ab_prev == nullptr) != (a.tab_prev == nullptr)) {
    return hipErrorInvalidValue;
  }
  // the chunks of a row block fastest: the workgroups in flight together
  // cover whole rows, as the column-chain sweep's do
  const dim3 grid((unsigned)nchunks, (unsigned)(a.ncols / kRChains), 1u);
  const int code = (a.in_f32 ? 2 : 0) | (a.out_f32 ? 1 : 0);
#define FPS_ROWS(TI, TO)                                                                          \
  do {                                                                                            \
    if (ev0 != nullptr)                                                                           \
      hipExtLaunchKernelGGL((k_sweep_rows<TI, TO>), grid, dim3(kRThreads), 0, st, ev0, ev1, 0, a); \
    else                                                                                          \
      hipLaunchKernelGGL((k_sweep_rows<TI, TO>), grid, dim3(kRThreads), 0, st, a);              \
  } while (0)
  switch (code) {
    case 0: FPS_ROWS(double, double); break;
    case 2: FPS_ROWS(float, double); break;
    case 3: FPS_ROWS(float, float); break;
    default: return hipErrorInvalidValue;  // a float output from a double input
  }
#undef FPS_ROWS
  return hipGetLastError();
}

}  // namespace fps
