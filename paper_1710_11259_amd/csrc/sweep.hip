// gfx950 kernels of the spectral Poisson solver.
//
// Sweep design (one launch per ADI half-sweep of Algorithm 2):
//   * every lane owns one chain and kSeg consecutive positions of it;
//     kWaves wavefronts stacked along the chain form a chunk.  Chains run
//     along the storage columns (k_sweep), or along the storage rows
//     (k_sweep_rows: the workgroup's 64 x 64 tile is read and written row
//     by row, one 64-position run per instruction, and turned around in LDS
//     on load and on store), with the same arithmetic: a row-chain pass on
//     an array equals a column-chain pass on its transpose bit for bit;
//   * the Thomas recurrences y_k = r_k - l_k y_{k-1} and
//     x_k = ib_k y_k - u_k x_{k+1} use factors of the whole chain (computed
//     once per shift on the host), so splitting a chain only re-associates
//     the recurrences: each piece runs with zero carries and the true carry
//     enters through precomputed multiplier products;
//   * carries between the segments of a chunk go through LDS; carries
//     between chunks are left in a small array, resolved by k_reduce
//     (reduce.hip), and folded into the next pass when it reads its input;
//   * the multiply by (A~ - p' I) that Algorithm 2 applies after each solve
//     along the same direction is r - (p + p') x, so no neighbour access is
//     needed; a column-chain pass can store its output transposed (the
//     batched form alternates column-chain passes on transposed arrays),
//     and the single-problem form alternates row- and column-chain passes
//     on one layout;
//   * the right-hand side G enters only the column half-step: the row
//     half-step's output V - G = R - 2p Y_{1/2} needs no G, and the column
//     half-step adds G to its right-hand side but not to its output.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

template <typename T>
__device__ __forceinline__ double ld_as_double(const T *p) {
  return (double)(*p);
}

// The right-hand side G is read once per ADI iteration and never written;
// non-temporal loads keep it from displacing, in the last-level cache, the
// array the previous half-step just wrote and this one reads (134 MB each at
// n = 4096).  Measured on the alternating pass pattern: 120 -> 86 us per
// pair of passes.
template <typename T>
__device__ __forceinline__ double ld_nt_as_double(const T *p) {
  return (double)__builtin_nontemporal_load(p);
}

// LDS of one sweep workgroup (doubles).  The early region holds the
// chunk's slice of the per-position tables, the producer's chunk carries of
// this workgroup's rows, the segment-carry combinations, the segment
// boundary values and (pre-multiplied passes) the stencil rows and the
// segment end values of the right-hand side; it is dead before the tile of
// the transposed store reuses the space.
constexpr int kSweepLds = kWaves * kCols * (kSeg + 1);  // also holds the 64 x 65 store tile
constexpr int kTabSlots = 5;                // l, ib, u, F1, Bk1
constexpr int OFF_TAB = 0;
constexpr int OFF_AB = OFF_TAB + kTabSlots * kChunk;
constexpr int OFF_L1 = OFF_AB + 2 * kChunk;
constexpr int OFF_SY = OFF_L1 + kL1;
constexpr int OFF_SX = OFF_SY + kWaves * kCols;
constexpr int OFF_PRE = OFF_SX + kWaves * kCols;   // stencil diagonal, coupling [2][kChunk]
constexpr int OFF_PF = OFF_PRE + 2 * kChunk;       // first rhs value of each segment
constexpr int OFF_PL = OFF_PF + kWaves * kCols;    // last rhs value of each segment
constexpr int OFF_END = OFF_PL + kWaves * kCols;
static_assert(OFF_END <= kSweepLds, "LDS carve-out");
constexpr int kThreads = kCols * kWaves;
constexpr int kTabN = kTabSlots * kChunk;
constexpr int kTabLoads = (kTabN + kThreads - 1) / kThreads;
static_assert(2 * kChunk <= kThreads && kL1 <= kThreads, "one carry / combination value per thread");
static_assert(T_L == 0 && T_IB == 1 && T_U == 2 && T_F1 == 3 && T_BK1 == 4, "table slot order");

// One workgroup unit of a sweep: chain block bx (64 chains) and chunk row
// by (parity-0 chunks first).
//   v   = in_scale * in + (chunk carries of the producing pass)
//   rhs = v + sg * g (kG == 1) or v;  kPre: rhs <- P rhs with the
//         tridiagonal stencil P (diagonal a.pre[r], coupling a.pre[npad + r]
//         of rows r and r + 1) applied along the chain;
//   x   = T^-1 rhs with T the pass's tridiagonal (tables);
//   out = x (out_mode 1, 3) or b - sigma x (out_mode 0, 2) with the output
//         base b = v + og * g (kG == 2) or v; modes 0 and 3 store transposed.
// kG selects how a g array enters: 0 none, 1 the right-hand side, 2 the
// output base (the two are kept apart to keep register pressure low).

// Geometry of the unit at chunk row `by` for wavefront w.
struct Unit {
  int s, c;
  int64_t mps, kc0, rbase, row0;
  bool active;
};

__device__ __forceinline__ Unit unit_of(const SweepArgs &a, int by, int w) {
  Unit u;
  u.s = by < a.nc0 ? 0 : 1;
  u.c = by - (u.s ? a.nc0 : 0);
  u.mps = u.s ? a.mp1 : a.mp0;
  u.kc0 = (int64_t)u.c * kChunk;
  u.active = u.kc0 + (int64_t)w * kSeg < u.mps;
  u.rbase = (u.s ? a.mp0 : 0) + u.kc0;
  u.row0 = u.rbase + (int64_t)w * kSeg;
  return u;
}

// Values of the chain block that do not depend on the chunk row: the
// producer's chunk index of these chains (as positions of its chains) and
// its carry vectors at those positions.
struct Cols {
  int64_t col0, col, cp;
  int sp;
  double bf, bk;
};

__device__ __forceinline__ Cols cols_of(const SweepArgs &a, int bx, int lane) {
  Cols q;
  q.col0 = (int64_t)bx * kCols;
  q.col = q.col0 + lane;
  q.sp = q.col0 >= a.mp0 ? 1 : 0;
  q.cp = (q.col0 - (q.sp ? a.mp0 : 0)) / kChunk;
  q.bf = q.bk = 0.0;
  if (a.tab_prev != nullptr) {
    const int64_t kp = q.col - (q.sp ? a.mp0 : 0);
    const double *tp = a.tab_prev + (int64_t)q.sp * kNTab * a.mstride;
    q.bf = tp[T_BF2 * a.mstride + kp];
    q.bk = tp[T_BK2 * a.mstride + kp];
  }
  return q;
}

// Component k (0: forward, 1: backward) of the producer's chunk carry of its
// chain r at chunk cp of parity sp, formed from its chunk boundary values
// for chains of at most two chunks: with one chunk there is no carry; with
// two, cf[1] = ylast[0] and cb[0] = xfirst[1] + BF2first[1] ylast[0] (the
// chunk-level recurrences of launch_reduce, cf[0] = cb[1] = 0).
__device__ __forceinline__ double fused_carry(const SweepArgs &a, int sp, int64_t cp, int64_t r,
                                              int k) {
  const int ncs = sp ? a.nc1 : a.nc0;
  if (ncs < 2 || (cp == 0) == (k == 0)) return 0.0;
  const int64_t nch = a.npad;
  const double y0 = a.lv_prev[((int64_t)(0 * 2 + sp) * 2 + 0) * nch + r];
  if (k == 0) return a.carry_scale * y0;
  const double x1 = a.lv_prev[((int64_t)(1 * 2 + sp) * 2 + 1) * nch + r];
  const double bf = a.ctab_prev[((int64_t)sp * kNCTab + C_BF2FIRST) * a.ncmax + 1];
  return a.carry_scale * (x1 + bf * y0);
}

// Per-unit small values, loaded before the unit's streaming loads without
// divergent branches (addresses are clamped), so that waiting for them does
// not wait for the streaming loads.
struct Small {
  double tv[kTabLoads];
  double l1v, abv, prv, prev_r, next_r, pe_before;
};

// This thread's value of the producer's chunk carries at the unit's
// positions (two per position, for the first 2 * kChunk threads).
__device__ __forceinline__ double load_abv(const SweepArgs &a, const Unit &u, const Cols &q,
                                           int tid) {
  if (a.tab_prev == nullptr) return 0.0;
  const int e2 = tid < 2 * kChunk ? tid : 2 * kChunk - 1;
  if (a.ctab_prev != nullptr) return fused_carry(a, q.sp, q.cp, u.rbase + (e2 >> 1), e2 & 1);
  return a.ab_prev[(((int64_t)q.sp * a.ncmax + q.cp) * a.npad + u.rbase) * 2 + e2];
}

template <typename Tin, typename Tg, int kG, bool kPre>
__device__ __forceinline__ void load_small(const SweepArgs &a, const Unit &u, const Cols &q,
                                           int tid, int w, Small &m) {
  const int64_t npad = a.npad, ms = a.mstride, ncmax = a.ncmax, ld = a.ld;
  const double *__restrict__ tab = a.tab + (int64_t)u.s * kNTab * ms + u.kc0;
#pragma unroll
  for (int k = 0; k < kTabLoads; ++k) {
    const int e = tid + k * kThreads < kTabN ? tid + k * kThreads : kTabN - 1;
    m.tv[k] = tab[(e / kChunk) * ms + (e % kChunk)];
  }
  m.l1v = a.l1[((int64_t)u.s * ncmax + u.c) * kL1 + (tid < kL1 ? tid : kL1 - 1)];
  m.abv = load_abv(a, u, q, tid);
  const bool has_prev = a.tab_prev != nullptr;
  m.prv = m.prev_r = m.next_r = m.pe_before = 0.0;
  if constexpr (kPre) {
    // The stencil rows of the chunk, and the right-hand side one row before
    // and one row after the chunk when those rows belong to the same chain.
    const Tin *__restrict__ in = (const Tin *)a.in;
    const Tg *__restrict__ gp = (const Tg *)a.g;
    const bool has_before = u.kc0 > 0, has_after = u.kc0 + kChunk < u.mps;
    const int e2 = tid < 2 * kChunk ? tid : 2 * kChunk - 1;
    m.prv = a.pre[(e2 / kChunk) * npad + u.rbase + (e2 % kChunk)];
    if (has_before) m.pe_before = a.pre[npad + u.rbase - 1];
    if ((w == 0 && has_before) || (w == kWaves - 1 && has_after)) {
      const int64_t r = w == 0 ? u.rbase - 1 : u.rbase + kChunk;
      double e0 = 0.0, e1 = 0.0;
      if (has_prev && a.ctab_prev != nullptr) {
        e0 = fused_carry(a, q.sp, q.cp, r, 0);
        e1 = fused_carry(a, q.sp, q.cp, r, 1);
      } else if (has_prev) {
        const double *ep = a.ab_prev + (((int64_t)q.sp * ncmax + q.cp) * npad + r) * 2;
        e0 = ep[0];
        e1 = ep[1];
      }
      double vr = a.in_scale * ld_as_double(in + r * ld + q.col) + e0 * q.bf + e1 * q.bk;
      if constexpr (kG == 1) vr += a.sg * ld_as_double(gp + r * ld + q.col);
      if (w == 0)
        m.prev_r = vr;
      else
        m.next_r = vr;
    }
  }
}

// Streaming loads (rows clamped for the idle segments past the chain end):
// v <- in, y <- g.
template <typename Tin, typename Tg, int kG>
__device__ __forceinline__ void load_stream(const SweepArgs &a, const Unit &u, const Cols &q,
                                            double *v, double *y) {
  const int64_t npad = a.npad, ld = a.ld;
  const Tin *__restrict__ in = (const Tin *)a.in;
#pragma unroll
  for (int i = 0; i < kSeg; ++i) {
    const int64_t r = u.row0 + i < npad ? u.row0 + i : npad - 1;
    v[i] = ld_as_double(in + r * ld + q.col);
  }
  if constexpr (kG != 0) {
    const Tg *__restrict__ gp = (const Tg *)a.g;
#pragma unroll
    for (int i = 0; i < kSeg; ++i) {
      const int64_t r = u.row0 + i < npad ? u.row0 + i : npad - 1;
      y[i] = ld_nt_as_double(gp + r * ld + q.col);
    }
  }
}

// Streaming loads of a row-chain unit (chains are the array's rows): wave w
// reads rows col0 + w * kSeg + i, one position per lane, so that every
// instruction moves one 64-position run of a row; compute_store turns the
// tile around in LDS.
template <typename Tin>
__device__ __forceinline__ void load_stream_rows(const SweepArgs &a, const Unit &u, const Cols &q,
                                                 int lane, int w, double *v) {
  const Tin *__restrict__ in = (const Tin *)a.in + (q.col0 + (int64_t)w * kSeg) * a.ld + u.rbase + lane;
#pragma unroll
  for (int i = 0; i < kSeg; ++i) v[i] = ld_as_double(in + i * a.ld);
}

// Elimination and store of one unit (lead_sync: synchronize before the LDS
// early region is written, for a workgroup that reuses its LDS).
template <typename Tin, typename Tg, typename Tout, int kG, bool kPre, bool kTL = false>
__device__ __forceinline__ void compute_store(const SweepArgs &a, const Unit &u, const Cols &q,
                                              const Small &m, double *v, double *y, double *lds,
                                              int tid, int lane, int w, bool lead_sync) {
  const int64_t ncols = a.ncols, ld = a.ld;
  const bool has_prev = a.tab_prev != nullptr;
  if (lead_sync) __syncthreads();
  if constexpr (kTL) {
    // Row chains: wave w holds rows (chains) w * kSeg + i with one position
    // per lane; after the turnaround lane holds chain `lane` at the
    // positions of segment w, as in the column-chain pass.
#pragma unroll
    for (int i = 0; i < kSeg; ++i) lds[(w * kSeg + i) * (kChunk + 1) + lane] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSeg; ++i) v[i] = lds[lane * (kChunk + 1) + w * kSeg + i];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kTabLoads; ++k)
    if (tid + k * kThreads < kTabN) lds[OFF_TAB + tid + k * kThreads] = m.tv[k];
  if (tid < kL1) lds[OFF_L1 + tid] = m.l1v;
  if (tid < 2 * kChunk) lds[OFF_AB + tid] = m.abv;
  if constexpr (kPre) {
    if (tid < 2 * kChunk) lds[OFF_PRE + tid] = m.prv;
  }
  __syncthreads();

  const double *Tl = lds + OFF_TAB + 0 * kChunk + w * kSeg;
  const double *Tib = lds + OFF_TAB + 1 * kChunk + w * kSeg;
  const double *Tu = lds + OFF_TAB + 2 * kChunk + w * kSeg;
  const double *Tf1 = lds + OFF_TAB + 3 * kChunk + w * kSeg;
  const double *Tbk1 = lds + OFF_TAB + 4 * kChunk + w * kSeg;
  const double *Ab = lds + OFF_AB + 2 * w * kSeg;

  // Right-hand side and output base.  Idle segments carry exact zeros.
  const double act = u.active ? 1.0 : 0.0;
  const double isc = act * a.in_scale;
  const double cA = has_prev ? act * q.bf : 0.0, cB = has_prev ? act * q.bk : 0.0;
#pragma unroll
  for (int i = 0; i < kSeg; ++i) {
    v[i] = isc * v[i] + Ab[2 * i] * cA + Ab[2 * i + 1] * cB;
    if constexpr (kG == 1) {
      y[i] = v[i] + (act * a.sg) * y[i];
    } else if constexpr (kG == 2) {
      const double gi = y[i];
      y[i] = v[i];
      v[i] += (act * a.og) * gi;
    } else {
      y[i] = v[i];
    }
  }
  if constexpr (kPre) {
    lds[OFF_PF + w * kCols + lane] = y[0];
    lds[OFF_PL + w * kCols + lane] = y[kSeg - 1];
    __syncthreads();
    const double ym = w > 0 ? lds[OFF_PL + (w - 1) * kCols + lane] : m.prev_r;
    const double yp = w < kWaves - 1 ? lds[OFF_PF + (w + 1) * kCols + lane] : m.next_r;
    const double *Pd = lds + OFF_PRE + w * kSeg;
    const double *Pe = lds + OFF_PRE + kChunk + w * kSeg;
    const double pem = w > 0 ? lds[OFF_PRE + kChunk + w * kSeg - 1] : m.pe_before;
    double t[kSeg];
#pragma unroll
    for (int i = 0; i < kSeg; ++i) {
      const double lo = i > 0 ? Pe[i - 1] * y[i - 1] : pem * ym;
      const double hi = i < kSeg - 1 ? Pe[i] * y[i + 1] : Pe[kSeg - 1] * yp;
      t[i] = (Pd[i] + a.pre_shift) * y[i] + lo + hi;
    }
#pragma unroll
    for (int i = 0; i < kSeg; ++i) y[i] = act * t[i];
  }

  // Forward elimination with zero carry-in, then the segment carry.
  {
    double carry = 0.0;
#pragma unroll
    for (int i = 0; i < kSeg; ++i) {
      y[i] = y[i] - Tl[i] * carry;
      carry = y[i];
    }
  }
  lds[OFF_SY + w * kCols + lane] = y[kSeg - 1];
  __syncthreads();
  double cf1 = 0.0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k)
    cf1 += lds[OFF_L1 + (0 * kWaves + w) * kWaves + k] * lds[OFF_SY + k * kCols + lane];
#pragma unroll
  for (int i = 0; i < kSeg; ++i) y[i] += Tf1[i] * cf1;
  const double ylast_chunk = y[kSeg - 1];

  // Backward substitution with zero carry-in, fused with the output.
  // Without a g term or stencil the right-hand side is recovered from the
  // forward values, r_k = y_k + l_k y_{k-1} (y_{-1} = cf1), so v need not
  // live on.
  constexpr bool kKeepV = kG != 0 || kPre;
  const double sigma = a.sigma;
  const bool out_x = a.out_mode == 1 || a.out_mode == 3;
  double xnext = 0.0, xfirst = 0.0;
#pragma unroll
  for (int i = kSeg - 1; i >= 0; --i) {
    const double x = y[i] * Tib[i] - Tu[i] * xnext;
    double rhs;
    if constexpr (kKeepV)
      rhs = v[i];
    else
      rhs = y[i] + Tl[i] * (i > 0 ? y[i - 1] : cf1);
    y[i] = out_x ? x : rhs - sigma * x;
    xnext = x;
    if (i == 0) xfirst = x;
  }
  lds[OFF_SX + w * kCols + lane] = xfirst;
  __syncthreads();
  double cb1 = 0.0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k)
    cb1 += lds[OFF_L1 + (1 * kWaves + w) * kWaves + k] * lds[OFF_SX + k * kCols + lane];
  const double coef = (out_x ? 1.0 : -sigma) * cb1;
#pragma unroll
  for (int i = 0; i < kSeg; ++i) y[i] += coef * Tbk1[i];

  // Chunk boundary values for the chunk carries.
  if (w == kWaves - 1) a.lv[(((int64_t)u.c * 2 + u.s) * 2 + 0) * ncols + q.col] = ylast_chunk;
  if (w == 0) a.lv[(((int64_t)u.c * 2 + u.s) * 2 + 1) * ncols + q.col] = xfirst + Tbk1[0] * cb1;

  Tout *__restrict__ out = (Tout *)a.out;
  if (a.out_mode == 1 || a.out_mode == 2) {
    if (u.active) {
#pragma unroll
      for (int i = 0; i < kSeg; ++i) out[(u.row0 + i) * ld + q.col] = (Tout)y[i];
    }
    return;
  }
  // Transposed store staged through LDS: the workgroup's 64 x 64 tile
  // (chain positions x chains) is transposed so that output row col0 + j
  // receives the chunk's 64 positions as one contiguous 512-byte run.
  static_assert(kChunk == kCols && kChunk * (kChunk + 1) <= kSweepLds, "store tile");
  __syncthreads();  // the early region is dead
#pragma unroll
  for (int i = 0; i < kSeg; ++i) lds[lane * (kChunk + 1) + w * kSeg + i] = y[i];
  __syncthreads();
  {
    // each wave stores kCols / kWaves output rows; 32 lanes per row, two
    // consecutive positions per lane
    constexpr int kRowsPerWave = kCols / kWaves;
#pragma unroll
    for (int t = 0; t < kRowsPerWave / 2; ++t) {
      const int orow = w * kRowsPerWave + 2 * t + (lane >> 5);
      const int pos = 2 * (lane & 31);
      const double v0 = lds[orow * (kChunk + 1) + pos];
      const double v1 = lds[orow * (kChunk + 1) + pos + 1];
      Tout *dst = out + (q.col0 + orow) * ld + u.rbase + pos;
      if constexpr (sizeof(Tout) == 8) {
        // one 16-byte store per lane: a row's 64 positions as one run
        // (pos even, rbase and ld multiples of 64)
        typedef double dbl2v __attribute__((ext_vector_type(2)));
        *(dbl2v *)dst = dbl2v{v0, v1};
      } else {
        typedef float flt2v __attribute__((ext_vector_type(2)));
        *(flt2v *)dst = flt2v{(float)v0, (float)v1};
      }
    }
  }
}

template <typename Tin, typename Tg, typename Tout, int kG, bool kPre, bool kTL = false>
__device__ __forceinline__ void sweep_block(const SweepArgs &a, const int bx, const int by,
                                            double *lds) {
  const int tid = threadIdx.x;
  const int lane = tid & (kCols - 1);
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const Cols q = cols_of(a, bx, lane);
  const Unit u = unit_of(a, by, w);
  Small m;
  load_small<Tin, Tg, kG, kPre>(a, u, q, tid, w, m);
  double v[kSeg], y[kSeg];
  if constexpr (kTL)
    load_stream_rows<Tin>(a, u, q, lane, w, v);
  else
    load_stream<Tin, Tg, kG>(a, u, q, v, y);
  compute_store<Tin, Tg, Tout, kG, kPre, kTL>(a, u, q, m, v, y, lds, tid, lane, w, false);
}

// Six wavefronts per SIMD (three workgroups per compute unit) fit every
// variant but the stencil pass with g in the output base, which would spill.
template <typename Tin, typename Tg, typename Tout, int kG, bool kPre>
__global__ __launch_bounds__(kCols *kWaves, (kPre && kG == 2) ? 4 : 6) void k_sweep(SweepArgs a) {
  __shared__ double lds[kSweepLds];
  if (blockIdx.z != 0) {
    const int64_t z = blockIdx.z;
    a.in = (const Tin *)a.in + z * a.bstride;
    if (kG != 0) a.g = (const Tg *)a.g + z * a.bstride;
    a.out = (Tout *)a.out + z * a.bstride;
    a.lv += z * a.lvb;
    if (a.tab_prev != nullptr && a.ctab_prev == nullptr) a.ab_prev += z * a.abb;
    if (a.ctab_prev != nullptr) a.lv_prev += z * a.lvb;
  }
  sweep_block<Tin, Tg, Tout, kG, kPre>(a, blockIdx.x + a.blk0, blockIdx.y + a.chk0, lds);
}

// Row-chain sweep (chains along the array's rows, stored in place of the
// input's layout): the column-chain arithmetic on tiles turned around in
// LDS on load and on store.  The chunks of a row block run fastest in the
// grid, so the workgroups in flight together cover whole rows.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kCols *kWaves, 6) void k_sweep_rows(SweepArgs a) {
  __shared__ double lds[kSweepLds];
  sweep_block<Tin, double, Tout, 0, false, true>(a, blockIdx.y + a.blk0, blockIdx.x + a.chk0, lds);
}

// Batched sweep: workgroup g belongs to problem wg_prob[g]; the problem's
// descriptor holds workspace offsets in place of its workspace pointers.
// kTL: row-chain problems (k_sweep_rows's arithmetic and layout; the
// descriptors carry out_mode 0 or 3, the row-wise stores).
template <typename Tin, typename Tg, typename Tout, int kG, bool kPre, bool kTL = false>
__global__ __launch_bounds__(kCols *kWaves, 6) void k_sweep_batch(const BatchSweep *__restrict__ d,
                                                                  const int *__restrict__ wg_prob,
                                                                  char *base, int wg_base) {
  __shared__ double lds[kSweepLds];
  const int g = (int)blockIdx.x + wg_base;
  const int k = __builtin_amdgcn_readfirstlane(wg_prob[g]);
  const BatchSweep &e = d[k];
  SweepArgs a = e.a;
  a.in = base + (intptr_t)a.in;
  if (kG != 0) a.g = base + (intptr_t)a.g;
  a.out = base + (intptr_t)a.out;
  a.lv = (double *)(base + (intptr_t)a.lv);
  if (a.ctab_prev != nullptr)
    a.lv_prev = (const double *)(base + (intptr_t)a.lv_prev);
  else if (a.tab_prev != nullptr)
    a.ab_prev = (const double *)(base + (intptr_t)a.ab_prev);
  const int local = g - e.wg_start;
  sweep_block<Tin, Tg, Tout, kG, kPre, kTL>(a, local % e.nbx, local / e.nbx, lds);
}

}  // namespace

// Launches one sweep (single: d == nullptr, grid from `a`; batched: `nwg`
// workgroups over the descriptors d) with the storage types of `a`.
struct SweepLaunch {
  const SweepArgs &a;
  const BatchSweep *d;
  const int *wg_prob;
  char *base;
  int nwg;
  hipStream_t st;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // optional: timestamps of this dispatch
  int wg_base = 0;
  template <typename Tin, typename Tg, typename Tout, int kG, bool kPre = false>
  void go() const {
    const int nch = a.nc0 + a.nc1;
    if (d == nullptr) {
      const int nbx = a.blk1 > 0 ? a.blk1 - a.blk0 : (int)(a.ncols / kCols);
      const int nby = a.chk1 > 0 ? a.chk1 - a.chk0 : nch;
      dim3 grid((unsigned)nbx, (unsigned)nby, (unsigned)(a.nbatch > 0 ? a.nbatch : 1));
      if (ev0 != nullptr)
        hipExtLaunchKernelGGL((k_sweep<Tin, Tg, Tout, kG, kPre>), grid, dim3(kCols * kWaves), 0, st,
                              ev0, ev1, 0, a);
      else
        hipLaunchKernelGGL((k_sweep<Tin, Tg, Tout, kG, kPre>), grid, dim3(kCols * kWaves), 0, st,
                           a);
    } else if constexpr (!kPre || kG != 2) {
      if (ev0 != nullptr)
        hipExtLaunchKernelGGL((k_sweep_batch<Tin, Tg, Tout, kG, kPre>), dim3((unsigned)nwg),
                              dim3(kCols * kWaves), 0, st, ev0, ev1, 0, d, wg_prob, base, wg_base);
      else
        hipLaunchKernelGGL((k_sweep_batch<Tin, Tg, Tout, kG, kPre>), dim3((unsigned)nwg),
                           dim3(kCols * kWaves), 0, st, d, wg_prob, base, wg_base);
    }
  }
};

hipError_t dispatch_sweep(const SweepLaunch &L, bool with_g) {
  const SweepArgs &a = L.a;
  const int code = (a.in_f32 ? 4 : 0) | (a.g_f32 ? 2 : 0) | (a.out_f32 ? 1 : 0);
  if (with_g && a.og != 0.0 && a.sg != 0.0) return hipErrorInvalidValue;
  const bool g_out = with_g && a.og != 0.0;
  if (a.pre != nullptr) {
    // stencil passes: float64 storage, or float storage without g (in/out
    // f/f) and with g in the right-hand side (f/f/f); batched ones without g
    // in the output
    if (L.d != nullptr && g_out) return hipErrorInvalidValue;
    if (code == 0) {
      if (!with_g)
        L.go<double, double, double, 0, true>();
      else if (g_out)
        L.go<double, double, double, 2, true>();
      else
        L.go<double, double, double, 1, true>();
    } else if (!with_g && (code & 5) == 5) {
      L.go<float, double, float, 0, true>();
    } else if (with_g && !g_out && code == 7) {
      L.go<float, float, float, 1, true>();
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (g_out) return hipErrorInvalidValue;  // g in the output base: stencil passes only
  if (!with_g) {
    switch (code & 5) {
      case 0: L.go<double, double, double, 0>(); break;
      case 4: L.go<float, double, double, 0>(); break;
      case 5: L.go<float, double, float, 0>(); break;
      default: return hipErrorInvalidValue;  // a float output from a double input
    }
  } else {
    switch (code) {
      case 0: L.go<double, double, double, 1>(); break;
      case 2: L.go<double, float, double, 1>(); break;
      case 6: L.go<float, float, double, 1>(); break;
      case 7: L.go<float, float, float, 1>(); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

// Chain-block and chunk-row ranges of a single launch: within the array,
// non-empty when given (blk0 = chk0 = 0 when not).
static bool ranges_ok(const SweepArgs &a) {
  const int64_t nbx = a.ncols / kCols, nch = a.nc0 + a.nc1;
  if (a.blk1 > 0 ? !(a.blk0 >= 0 && a.blk0 < a.blk1 && a.blk1 <= nbx) : a.blk0 != 0) return false;
  if (a.chk1 > 0 ? !(a.chk0 >= 0 && a.chk0 < a.chk1 && a.chk1 <= nch) : a.chk0 != 0) return false;
  return true;
}

hipError_t launch_sweep(const SweepArgs &a, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int nchunks = a.nc0 + a.nc1;
  if (a.npad % kCols != 0 || a.ncols % kCols != 0 || nchunks <= 0 || a.in == nullptr)
    return hipErrorInvalidValue;
  if (!ranges_ok(a)) return hipErrorInvalidValue;
  if (a.ctab_prev != nullptr) {  // carries formed in the sweep: at most two chunks per chain
    if (a.tab_prev == nullptr || a.lv_prev == nullptr || a.ncmax > 2) return hipErrorInvalidValue;
  } else if ((a.ab_prev == nullptr) != (a.tab_prev == nullptr)) {
    return hipErrorInvalidValue;
  }
  if ((a.out_mode == 0 || a.out_mode == 3) && (a.ncols != a.npad || a.ld != a.npad))
    return hipErrorInvalidValue;
  if (a.out_mode < 0 || a.out_mode > 3) return hipErrorInvalidValue;
  if (a.ld < a.ncols) return hipErrorInvalidValue;
  return dispatch_sweep(SweepLaunch{a, nullptr, nullptr, nullptr, 0, st, ev0, ev1}, a.g != nullptr);
}

hipError_t launch_sweep_rows(const SweepArgs &a0, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int nchunks = a0.nc0 + a0.nc1;
  if (a0.npad % kCols != 0 || a0.ncols % kCols != 0 || nchunks <= 0 || a0.in == nullptr ||
      a0.out == nullptr)
    return hipErrorInvalidValue;
  if (a0.ncols != a0.npad || a0.ld < a0.npad || a0.ld % 4 != 0) return hipErrorInvalidValue;
  if (a0.out_mode != 1 && a0.out_mode != 2) return hipErrorInvalidValue;
  if (a0.g != nullptr || a0.pre != nullptr || a0.nbatch > 1) return hipErrorInvalidValue;
  if (a0.ctab_prev != nullptr) {
    if (a0.tab_prev == nullptr || a0.lv_prev == nullptr || a0.ncmax > 2) return hipErrorInvalidValue;
  } else if ((a0.ab_prev == nullptr) != (a0.tab_prev == nullptr)) {
    return hipErrorInvalidValue;
  }
  if (!ranges_ok(a0)) return hipErrorInvalidValue;
  SweepArgs a = a0;
  a.out_mode = a0.out_mode == 1 ? 3 : 0;  // the same outputs, stored along rows
  const int nbx = a.blk1 > 0 ? a.blk1 - a.blk0 : (int)(a.ncols / kCols);
  const int nby = a.chk1 > 0 ? a.chk1 - a.chk0 : nchunks;
  const dim3 grid((unsigned)nby, (unsigned)nbx, 1u);
  const int code = (a.in_f32 ? 2 : 0) | (a.out_f32 ? 1 : 0);
#define FPS_ROWS(TI, TO)                                                                         \
  do {                                                                                           \
    if (ev0 != nullptr)                                                                          \
      hipExtLaunchKernelGGL((k_sweep_rows<TI, TO>), grid, dim3(kCols * kWaves), 0, st, ev0, ev1, \
                            0, a);                                                               \
    else                                                                                         \
      hipLaunchKernelGGL((k_sweep_rows<TI, TO>), grid, dim3(kCols * kWaves), 0, st, a);          \
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

hipError_t launch_sweep_batch_rows(const SweepArgs &types, const BatchSweep *d, const int *wg_prob,
                                   int nwg, char *base, hipStream_t st, int wg_base, hipEvent_t ev0,
                                   hipEvent_t ev1) {
  if (nwg <= 0) return hipSuccess;
  if (types.blk1 != 0 || types.chk1 != 0 || types.pre != nullptr) return hipErrorInvalidValue;
  const int code = (types.in_f32 ? 2 : 0) | (types.out_f32 ? 1 : 0);
  const dim3 grid((unsigned)nwg), block(kCols * kWaves);
#define FPS_BROWS(TI, TO)                                                                        \
  do {                                                                                           \
    if (ev0 != nullptr)                                                                          \
      hipExtLaunchKernelGGL((k_sweep_batch<TI, double, TO, 0, false, true>), grid, block, 0, st, \
                            ev0, ev1, 0, d, wg_prob, base, wg_base);                             \
    else                                                                                         \
      hipLaunchKernelGGL((k_sweep_batch<TI, double, TO, 0, false, true>), grid, block, 0, st, d, \
                         wg_prob, base, wg_base);                                                \
  } while (0)
  switch (code) {
    case 0: FPS_BROWS(double, double); break;
    case 2: FPS_BROWS(float, double); break;
    case 3: FPS_BROWS(float, float); break;
    default: return hipErrorInvalidValue;
  }
#undef FPS_BROWS
  return hipGetLastError();
}

hipError_t launch_sweep_batch(const SweepArgs &types, bool with_g, const BatchSweep *d,
                              const int *wg_prob, int nwg, char *base, hipStream_t st,
                              int wg_base, hipEvent_t ev0, hipEvent_t ev1) {
  if (nwg <= 0) return hipSuccess;
  if (types.blk1 != 0 || types.chk1 != 0) return hipErrorInvalidValue;  // whole problems only
  return dispatch_sweep(SweepLaunch{types, d, wg_prob, base, nwg, st, ev0, ev1, wg_base}, with_g);
}

}  // namespace fps
