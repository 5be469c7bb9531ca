// gfx950 LDS-resident ADI for the z-eigenbasis cube: every z-slice of the
// eigen-transformed system is a Sylvester equation of its own, and since A~
// is block diagonal by parity, each slice splits again into four
// independent problems, one per (y parity, x parity) block of at most
// 128 x 128 unknowns for n <= 256.  One workgroup keeps such a block in LDS
// (and the right-hand side in registers) for all the slice's ADI steps of
// Algorithm 2, so the iteration reads G^ once and writes Y^ once instead of
// streaming three arrays through HBM per step.
//
// Per step j the pass form of the batched slice sweeps (the same tables,
// shifts and stencil):
//   x solve along the block's rows:    v <- v - s1 T1^-1 v,
//   y solve along its columns:         v <- v - s2 T2^-1 P (v - G)
//                                      (the last step keeps T2^-1 P (v - G)),
// with T1, T2 the slice's shifted tridiagonals (whole-chain Thomas factors
// of the plan's tables) and P = A~ + mu the stencil.  The nested cube's
// inner ADI on every z-slice is the same loop with the stencil A~ in both
// solves (x solve: v <- v - s1 T1^-1 A~ v; the last y solve keeps it).  Each chain of up to
// 128 positions is split into eight chunks of 16, one per thread: all solve
// with zero carries, exchange their boundary values through LDS, and add
// the carries through the chunk vectors BF2 / Bk2 of 16-position chunks
// after the chunk-level recurrences (those of the sweeps' carry kernel).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

constexpr int kLB = 128;             // largest parity block (chain length)
constexpr int kLQ = 8;               // chunks per chain (threads per chain)
constexpr int kLH = kLB / kLQ;       // positions per thread (one chunk)
constexpr int kLP = kLB + 2;         // LDS row pitch in doubles (16-byte rows)
constexpr int kLThreads = kLQ * kLB;  // 1024
static_assert(kLH == kZeigLdsChunk, "chunk tables of the plan");

// Per-solve tables staged in LDS: l, ib, u, BF2, Bk2 at every position,
// then F2last, BF2first, Bk2first of every chunk.
constexpr int kNT = 5;
constexpr int kTabSolve = kNT * kLB + 3 * kLQ;
static_assert(T_L == 0 && T_IB == 1 && T_U == 2, "slots kept");

struct Ends {
  double ylast, xfirst;
};
typedef double dbl2 __attribute__((ext_vector_type(2)));

// One chain chunk in registers: the Thomas recurrences with zero carries
// over positions k0 .. k1-1 (tables tl, tib, tu in LDS at the chain's
// positions, 16-byte aligned, readable up to k0 + kLH - 1); r holds the
// chunk's right-hand side on entry and its chunk-local solution on return.
// Each pass reads its table values into registers ahead of its recurrence.
// kFull: the chunk has all kLH positions (no guards).
template <bool kFull>
__device__ __forceinline__ Ends chunk_solve(double (&r)[kLH], int k0, int k1, const double *tl,
                                            const double *tib, const double *tu) {
  // bursts of kB positions: their table values are read together, and
  // scheduling barriers keep the compiler from hoisting several bursts at
  // once (they would not fit the registers of two wavefronts per SIMD)
  constexpr int kB = 8;
  double yp = 0.0;
#pragma unroll
  for (int b0 = 0; b0 < kLH; b0 += kB) {
    __builtin_amdgcn_sched_barrier(0);
    double t[kB];
#pragma unroll
    for (int i = 0; i < kB; i += 2) {
      const dbl2 q = *(const dbl2 *)(tl + k0 + b0 + i);
      t[i] = q.x;
      t[i + 1] = q.y;
    }
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      if (kFull || k0 + b0 + i < k1) {
        r[b0 + i] = r[b0 + i] - t[i] * yp;
        yp = r[b0 + i];
      }
    }
  }
  double xn = 0.0, xf = 0.0;
#pragma unroll
  for (int b0 = kLH - kB; b0 >= 0; b0 -= kB) {
    __builtin_amdgcn_sched_barrier(0);
    double ib[kB], u[kB];
#pragma unroll
    for (int i = 0; i < kB; i += 2) {
      const dbl2 qi = *(const dbl2 *)(tib + k0 + b0 + i);
      const dbl2 qu = *(const dbl2 *)(tu + k0 + b0 + i);
      ib[i] = qi.x;
      ib[i + 1] = qi.y;
      u[i] = qu.x;
      u[i + 1] = qu.y;
    }
#pragma unroll
    for (int i = kB - 1; i >= 0; --i) {
      if (kFull || k0 + b0 + i < k1) {
        r[b0 + i] = r[b0 + i] * ib[i] - u[i] * xn;
        xn = r[b0 + i];
        xf = r[b0 + i];
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  return Ends{yp, xf};
}

// The carries into every chunk of chain ch (nq chunks) from the chunks'
// boundary values (ey, ex: [chunk][chain] in LDS) and the chunk table C
// (F2last, BF2first, Bk2first by chunk), written back in place: ey[c][ch]
// <- cf(c), ex[c][ch] <- cb(c), with
//   cf(0) = 0, cf(c+1) = F2last(c) cf(c) + ylast(c),
//   cb(nq-1) = 0, cb(c) = Bk2first(c+1) cb(c+1) + xfirst(c+1) + BF2first(c+1) cf(c+1).
__device__ __forceinline__ void chain_carries(double (*ey)[kLB], double (*ex)[kLB],
                                              const double *C, int ch, int nq) {
  double f[kLQ], b[kLQ];
  f[0] = 0.0;
#pragma unroll
  for (int c = 0; c + 1 < kLQ; ++c) f[c + 1] = c + 1 < nq ? C[c] * f[c] + ey[c][ch] : 0.0;
  b[kLQ - 1] = 0.0;
#pragma unroll
  for (int c = kLQ - 2; c >= 0; --c)
    b[c] = c + 1 < nq ? C[2 * kLQ + c + 1] * b[c + 1] + (ex[c + 1][ch] + C[kLQ + c + 1] * f[c + 1])
                      : 0.0;
#pragma unroll
  for (int c = 0; c < kLQ; ++c) {
    ey[c][ch] = f[c];
    ex[c][ch] = b[c];
  }
}

// The two halves of one thread's part of a solve (a barrier and the
// boundary-value exchange between them).  x solve: chain cells cell[i]
// (row), right-hand side v; y solve: cells cell[i * kLP] (column),
// right-hand side P (v - G) (v - G at the last step).  kFull: a full chunk.
// kSt: the right-hand side is P v with the stencil along the row (diagonal
// and coupling of position k at Px[k * kLP], Px[k * kLP + 1]; v before and
// after the chunk wlo, whi, zero past the chain).
template <bool kFull, bool kSt = false>
__device__ __forceinline__ Ends x_local(double (&r)[kLH], const double *cell, int k0, int k1,
                                        const double *T, const double *Px = nullptr,
                                        double wlo = 0.0, double whi = 0.0) {
  if constexpr (kFull) {  // 16-byte reads of the row (cell 16-byte aligned)
#pragma unroll
    for (int i = 0; i < kLH; i += 2) {
      const dbl2 p = *(const dbl2 *)(cell + i);
      r[i] = p.x;
      r[i + 1] = p.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kLH; ++i) r[i] = k0 + i < k1 ? cell[i] : 0.0;
  }
  if constexpr (kSt) {
    // rhs_k = d_k v_k + e_{k-1} v_{k-1} + e_k v_{k+1}
    double wm = wlo;
#pragma unroll
    for (int i = 0; i < kLH; ++i) {
      const int k = k0 + i;
      if (kFull || k < k1) {
        const double w = r[i];
        const double wp = i + 1 < kLH ? r[i + 1] : whi;
        const double lo = k > 0 ? Px[(k - 1) * kLP + 1] * wm : 0.0;
        const double hi = Px[k * kLP + 1] * wp;
        r[i] = (Px[k * kLP] + 0.0) * w + lo + hi;
        wm = w;
      }
    }
  }
  return chunk_solve<kFull>(r, k0, k1, T, T + kLB, T + 2 * kLB);
}

template <bool kFull>
__device__ __forceinline__ void x_out(const double (&r)[kLH], double *cell, int k0, int k1,
                                      const double *T, double cf, double cb, double s1) {
  const double *bf2 = T + 3 * kLB, *bk2 = T + 4 * kLB;
  // the cells still hold the input v
  if constexpr (kFull) {
#pragma unroll
    for (int i = 0; i < kLH; i += 2) {
      const dbl2 v = *(const dbl2 *)(cell + i);
      const dbl2 f2 = *(const dbl2 *)(bf2 + k0 + i), b2 = *(const dbl2 *)(bk2 + k0 + i);
      *(dbl2 *)(cell + i) = dbl2{v.x - s1 * (r[i] + (cf * f2.x + cb * b2.x)),
                                 v.y - s1 * (r[i + 1] + (cf * f2.y + cb * b2.y))};
    }
  } else {
#pragma unroll
    for (int i = 0; i < kLH; ++i) {
      const int k = k0 + i;
      if (k < k1) cell[i] = cell[i] - s1 * (r[i] + (cf * bf2[k] + cb * bk2[k]));
    }
  }
}

template <bool kFull>
__device__ __forceinline__ Ends y_local(double (&r)[kLH], const double *cell, const double *gc,
                                        int k0, int k1, const double *T, const double *Pd,
                                        const double *Pe, double mu, double wlo, double whi,
                                        bool nost) {
  // w = v - G (the cells keep v until after the barrier that follows)
#pragma unroll
  for (int i = 0; i < kLH; ++i) r[i] = (kFull || k0 + i < k1) ? cell[i * kLP] - gc[i] : 0.0;
  if (!nost) {
    // rhs_k = (d_k + mu) w_k + e_{k-1} w_{k-1} + e_k w_{k+1}
    double wm = wlo;
#pragma unroll
    for (int i = 0; i < kLH; ++i) {
      const int k = k0 + i;
      if (kFull || k < k1) {
        const double w = r[i];
        const double wp = i + 1 < kLH ? r[i + 1] : whi;
        const double lo = k > 0 ? Pe[k - 1] * wm : 0.0;
        const double hi = Pe[k] * wp;
        r[i] = (Pd[k] + mu) * w + lo + hi;
        wm = w;
      }
    }
  }
  return chunk_solve<kFull>(r, k0, k1, T, T + kLB, T + 2 * kLB);
}

template <bool kFull>
__device__ __forceinline__ void y_out(const double (&r)[kLH], double *cell, int k0, int k1,
                                      const double *T, double cf, double cb, double s2,
                                      bool last) {
  const double *bf2 = T + 3 * kLB, *bk2 = T + 4 * kLB;
#pragma unroll
  for (int i = 0; i < kLH; ++i) {
    const int k = k0 + i;
    if (kFull || k < k1) {
      const double x = r[i] + (cf * bf2[k] + cb * bk2[k]);
      cell[i * kLP] = last ? x : cell[i * kLP] - s2 * x;
    }
  }
}

// Workgroup g: sorted slice g / 4 (J descending, inactive slices last),
// block (sy, sx) = ((g / 2) % 2, g % 2).  Threads: chain t % 128, chunk
// t / 128 (two wavefronts per chunk, four per SIMD).  The next step's tables are fetched
// into registers while a step runs; each solve's LDS tables are replaced
// right after that solve's last read.  kNested: the nested cube's inner ADI
// (stencil in both solves, kept at the last step; the row padding of Yb
// holds the stencil of the x parity; output +(the final y solve)).
template <bool kNested>
__global__ __launch_bounds__(kLThreads, 1) void k_zeig_lds(ZeigLdsArgs a) {
  __shared__ __align__(16) double Yb[kLB * kLP];
  __shared__ double ey[kLQ][kLB], exf[kLQ][kLB];  // chunk boundary values
  __shared__ __align__(16) double Tb[2][kTabSolve];  // [x / y solve]
  __shared__ double Pd[kLB], Pe[kLB];  // A~ along the y parity: diagonal, coupling
  const int g = blockIdx.x;
  const int kk = g >> 2, sy = (g >> 1) & 1, sx = g & 1;
  const int tid = threadIdx.x;
  const int ch = tid & (kLB - 1);
  const int q = __builtin_amdgcn_readfirstlane(tid >> 7);
  const int64_t npad = a.npad, mp0 = a.mp0, ms = a.mstride, nq32 = a.mstride / kLH;
  const int my = sy ? a.m1 : a.m0, mx = sx ? a.m1 : a.m0;
  const int64_t mpy = sy ? npad - mp0 : mp0, mpx = sx ? npad - mp0 : mp0;
  const int64_t r0 = sy ? mp0 : 0, c0 = sx ? mp0 : 0;
  const int slice = kNested ? kk : a.slice[kk], J = kNested ? a.J_all : a.J[kk];
  const double *__restrict__ Gs = a.G + ((int64_t)slice * npad + r0) * npad + c0;
  double *__restrict__ Ys = a.Y + ((int64_t)slice * npad + r0) * npad + c0;

  if (J == 0 || my == 0 || mx == 0) {  // uniform: the block of Y^ is zero
    for (int64_t y = tid / 64; y < mpy; y += kLThreads / 64)
      for (int64_t x = tid % 64; x < mpx; x += 64) Ys[y * npad + x] = 0.0;
    return;
  }
  const int tab0 = kNested ? a.tab0_all : a.tab0[kk];
  // step j: x solve on table tab0 + kTs j, y solve on tab0 + kTs j + kTy
  constexpr int kTs = kNested ? 1 : 2, kTy = kNested ? 0 : 1;
  // Step j's tables are fetched in 64-value pieces, one per (wavefront,
  // round p): piece z = p * 16 + wavefront is piece z % 11 of solve z / 11
  // (0: x, 1: y), either half (z % 11) % 2 of position table (z % 11) / 2 (l,
  // ib, u from the plan's tables, BF2, Bk2 from the kernel's chunk tables) or,
  // for z % 11 == 10, the chunk table (kind, chunk) = (lane / 8, lane % 8).
  // Which table a piece reads, and its stride per step, are uniform over the
  // wavefront; a lane keeps its offset, the value in flight and whether it
  // lies before the chain's end (zero past it).
  constexpr int kWaves = kLThreads / 64;
  constexpr int kPieces = 2 * kNT + 1;
  constexpr int kRounds = (2 * kPieces + kWaves - 1) / kWaves;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  double tv[kRounds];
  const double *src[kRounds];
  int64_t step[kRounds];
  int off[kRounds], dst[kRounds], psv[kRounds];
  bool live[kRounds];
#pragma unroll
  for (int p = 0; p < kRounds; ++p) {
    const int z = p * kWaves + wv;
    const bool act = z < 2 * kPieces;
    const int sv = z >= kPieces ? 1 : 0, r = z - sv * kPieces;
    const int s = sv ? sy : sx, m = sv ? my : mx;
    const int64_t t = tab0 + kTy * sv;  // the table of step 0
    psv[p] = sv;
    if (r < 2 * kNT) {
      const int row = r >> 1, k = (r & 1) * 64 + lane;
      src[p] = row < 3 ? a.tab + ((t * 2 + s) * kNTab + row) * ms
                       : a.tab32 + ((t * 2 + s) * 2 + (row - 3)) * ms;
      step[p] = kTs * (row < 3 ? 2 * kNTab * ms : 4 * ms);
      off[p] = k;
      live[p] = act && k < m;
      dst[p] = act ? sv * kTabSolve + row * kLB + k : -1;
    } else {
      const int kind = lane >> 3, c = lane & 7;
      src[p] = a.ctab32 + (t * 2 + s) * 3 * nq32;
      step[p] = kTs * 6 * nq32;
      off[p] = kind * (int)nq32 + c;
      live[p] = act && lane < 3 * kLQ && c * kLH < m;
      dst[p] = act && lane < 3 * kLQ ? sv * kTabSolve + kNT * kLB + lane : -1;
    }
  }
  // step j's tables (called with j = 0, 1, 2, ... in turn)
  auto fetch = [&](int) {
#pragma unroll
    for (int p = 0; p < kRounds; ++p) {
      tv[p] = live[p] ? src[p][off[p]] : 0.0;
      src[p] += step[p];
    }
  };
  // stores the fetched values of solve sv
  auto stash = [&](int sv) {
#pragma unroll
    for (int p = 0; p < kRounds; ++p)
      if (psv[p] == sv && dst[p] >= 0) (&Tb[0][0])[dst[p]] = tv[p];
  };
  fetch(0);
  // G^ block into LDS (rows y < my, columns x < mx), coalesced by row; the
  // stencil of the y parity.
  for (int y = tid / kLB; y < my; y += kLThreads / kLB)
    if (ch < mx) Yb[y * kLP + ch] = Gs[(int64_t)y * npad + ch];
  if (tid < kLB) {
    Pd[tid] = tid < my ? a.pre[r0 + tid] : 0.0;
    Pe[tid] = tid < my ? a.pre[npad + r0 + tid] : 0.0;
    if constexpr (kNested) {  // the x parity's stencil in the row padding
      Yb[tid * kLP + kLB] = tid < mx ? a.pre[c0 + tid] : 0.0;
      Yb[tid * kLP + kLB + 1] = tid < mx ? a.pre[npad + c0 + tid] : 0.0;
    }
  }
  // This thread's column chunk of G^ for every y solve, and the halo values
  // of the neighbouring chunks (the stencil couples the chunks' ends).
  const int ky0 = q * kLH, ky1 = ky0 + kLH < my ? ky0 + kLH : my;
  const int kx0 = q * kLH, kx1 = kx0 + kLH < mx ? kx0 + kLH : mx;
  const int nqy = (my + kLH - 1) / kLH, nqx = (mx + kLH - 1) / kLH;
  const bool fullx = kx1 - kx0 == kLH, fully = ky1 - ky0 == kLH;  // uniform per wavefront
  double gc[kLH];
#pragma unroll
  for (int i = 0; i < kLH; ++i)
    gc[i] = (ch < mx && ky0 + i < ky1) ? Gs[(int64_t)(ky0 + i) * npad + ch] : 0.0;
  const bool hlo = ky0 > 0 && ky0 <= my, hhi = ky1 < my;
  const double glo = (ch < mx && hlo) ? Gs[(int64_t)(ky0 - 1) * npad + ch] : 0.0;
  const double ghi = (ch < mx && hhi) ? Gs[(int64_t)ky1 * npad + ch] : 0.0;
  stash(0);
  stash(1);
  __syncthreads();

  const double mu = kNested ? 0.0 : a.mu[kk];
  const double *__restrict__ sig = kNested ? a.sig : a.sig + a.sig0[kk];
  double r[kLH];
  for (int j = 0; j < J; ++j) {
    const bool last = j == J - 1;
    const double s1 = sig[2 * j], s2 = sig[2 * j + 1];
    if (!last) fetch(j + 1);
    // ---- x solve: chain = row ch (positions x), chunk q; tables of parity sx
    {
      const double *T = Tb[0];
      const bool on = ch < my && kx0 < mx;
      double *cell = Yb + ch * kLP + kx0;
      if (on) {
        Ends e;
        if constexpr (kNested) {
          const double wlo = kx0 > 0 ? cell[-1] : 0.0, whi = kx1 < mx ? cell[kx1 - kx0] : 0.0;
          e = fullx ? x_local<true, true>(r, cell, kx0, kx1, T, Yb + kLB, wlo, whi)
                    : x_local<false, true>(r, cell, kx0, kx1, T, Yb + kLB, wlo, whi);
        } else {
          e = fullx ? x_local<true>(r, cell, kx0, kx1, T) : x_local<false>(r, cell, kx0, kx1, T);
        }
        ey[q][ch] = e.ylast;
        exf[q][ch] = e.xfirst;
      }
      __syncthreads();
      // the carries of every chunk of the row, once per chain
      if (q == 0 && ch < my) chain_carries(ey, exf, T + kNT * kLB, ch, nqx);
      __syncthreads();
      if (on) {
        const double cf = ey[q][ch], cb = exf[q][ch];
        if (fullx)
          x_out<true>(r, cell, kx0, kx1, T, cf, cb, s1);
        else
          x_out<false>(r, cell, kx0, kx1, T, cf, cb, s1);
      }
      __syncthreads();
      if (!last) stash(0);  // the x tables were last read above
    }
    // ---- y solve: chain = column ch (positions y), chunk q; tables of
    // parity sy; right-hand side P (v - G) with P = A~ + mu (the identity at
    // the last step)
    {
      const double *T = Tb[1];
      const bool on = ch < mx && ky0 < my;
      double *cell = Yb + ky0 * kLP + ch;
      if (on) {
        const double wlo = hlo ? Yb[(ky0 - 1) * kLP + ch] - glo : 0.0;
        const double whi = hhi ? Yb[ky1 * kLP + ch] - ghi : 0.0;
        const Ends e =
            fully ? y_local<true>(r, cell, gc, ky0, ky1, T, Pd, Pe, mu, wlo, whi, last && !kNested)
                  : y_local<false>(r, cell, gc, ky0, ky1, T, Pd, Pe, mu, wlo, whi, last && !kNested);
        ey[q][ch] = e.ylast;
        exf[q][ch] = e.xfirst;
      }
      __syncthreads();
      // the carries of every chunk of the column, once per chain
      if (q == 0 && ch < mx) chain_carries(ey, exf, T + kNT * kLB, ch, nqy);
      __syncthreads();
      if (on) {
        const double cf = ey[q][ch], cb = exf[q][ch];
        if (fully)
          y_out<true>(r, cell, ky0, ky1, T, cf, cb, s2, last);
        else
          y_out<false>(r, cell, ky0, ky1, T, cf, cb, s2, last);
      }
      __syncthreads();
      if (!last) stash(1);  // the y tables were last read above
    }
  }
  // Y^ block = -(the last y solve), zero on the padding; kNested: cy x +
  // cr G + cb B (the outer step's update of the nested cube), in that order.
  if constexpr (kNested) {
    const double *__restrict__ Bs =
        a.B ? a.B + ((int64_t)slice * npad + r0) * npad + c0 : nullptr;
    for (int64_t y = tid / 64; y < mpy; y += kLThreads / 64)
      for (int64_t x = tid % 64; x < mpx; x += 64) {
        double v = (y < my && x < mx) ? Yb[y * kLP + x] : 0.0;
        v = a.cy * v;
        if (Bs) {  // null: the last outer step stores x itself
          v += a.cr * Gs[y * npad + x];
          v += a.cb * Bs[y * npad + x];
        }
        Ys[y * npad + x] = v;
      }
  } else {
    for (int64_t y = tid / 64; y < mpy; y += kLThreads / 64)
      for (int64_t x = tid % 64; x < mpx; x += 64)
        Ys[y * npad + x] = (y < my && x < mx) ? -Yb[y * kLP + x] : 0.0;
  }
}

}  // namespace

bool zeig_lds_fits(int64_t m0, int64_t m1) { return m0 <= kLB && m1 <= kLB; }

hipError_t launch_zeig_lds(const ZeigLdsArgs &a, int nslices, hipStream_t st, hipEvent_t ev0,
                           hipEvent_t ev1, bool nested) {
  if (nslices <= 0) return hipSuccess;
  if (!zeig_lds_fits(a.m0, a.m1) || a.mp0 > kLB || a.npad - a.mp0 > kLB ||
      a.mstride % kLH != 0 || a.tab32 == nullptr || a.ctab32 == nullptr)
    return hipErrorInvalidValue;
  if (nested ? (a.tab0_all < 0 || a.J_all < 1 || a.sig == nullptr || nslices > a.npad)
             : (a.slice == nullptr || a.J == nullptr || a.tab0 == nullptr || a.sig0 == nullptr ||
                a.mu == nullptr))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)(4 * nslices)), block(kLThreads);
  auto k = nested ? k_zeig_lds<true> : k_zeig_lds<false>;
  if (ev0 != nullptr)
    hipExtLaunchKernelGGL(k, grid, block, 0, st, ev0, ev1, 0, a);
  else
    hipLaunchKernelGGL(k, grid, block, 0, st, a);
  return hipGetLastError();
}

}  // namespace fps
