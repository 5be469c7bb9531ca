// Launch interfaces of the gfx950 kernels of the spectral Poisson solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "planner.hpp"

namespace fps {

// One ADI half-sweep over a parity-blocked npad x npad array whose chains
// run down the storage rows (one chain per storage column).
//   input  v = in_scale * in (+ carry correction of the producing pass)
//   solve  x = (A~ + p I)^-1 r along each chain (per parity), r = v + sg * g
//          (r = v when g is null)
//   output out = v - sigma x   (stored transposed), or x itself (final,
//          stored in place orientation).  Chunk-level carries are not applied
//          by the producer: it leaves its chunk boundary values in `lv`;
//          launch_reduce turns them into carries, which the consumer (the
//          next sweep, or launch_finalize after the last one) folds in.
struct SweepArgs {
  const void *in;          // [npad*npad], storage type in_f32
  double in_scale;
  const double *ab_prev;   // producer's chunk carries [2][ncmax][npad][2], or null
  const double *tab_prev;  // producer's per-position tables (its shift) [2][kNTab][mstride]
  const void *g;           // [npad*npad] G term (same orientation as `in`) or nullptr
  double sg;
  const double *tab;       // this pass's tables [2][kNTab][mstride]
  const double *l1;        // this pass's segment-carry combinations [2][ncmax][kL1]
  double sigma;
  void *out;               // [npad*npad], storage type out_f32
  double *lv;              // chunk boundary values [ncmax][2][2][npad]
  int final_mode;          // 1: out = x, not transposed
  int64_t npad, mp0, mp1, mstride, ncmax;
  int nc0, nc1;
  // Storage types (0: double, 1: float; arithmetic is double throughout).
  // Supported: without g, in/out = d/d, f/d, f/f; with g, in/g/out =
  // d/d/d, d/f/d, f/f/d, f/f/f.
  int in_f32, g_f32, out_f32;
};

hipError_t launch_sweep(const SweepArgs &a, hipStream_t st);

// Batched sweeps over several independent problems in one launch.  The
// workspace pointers of each descriptor's SweepArgs (in, g, out, lv,
// ab_prev) hold byte offsets from `base`; tab, tab_prev and l1 are device
// pointers; ab_prev is used iff tab_prev is non-null.  Workgroup g runs
// block (local % nbx, local / nbx), local = g - wg_start, of problem
// wg_prob[g].  Storage types and the presence of g come from `types` /
// `with_g` and must be those of every descriptor.
struct BatchSweep {
  SweepArgs a;
  int wg_start, nbx;
};
hipError_t launch_sweep_batch(const SweepArgs &types, bool with_g, const BatchSweep *d,
                              const int *wg_prob, int nwg, char *base, hipStream_t st);

// Chunk carries: for every chain, the forward and backward carry into each
// chunk, scaled by `scale`, into ab [2][ncmax][npad][2] (comb: the carry
// combinations of the producing pass's shift).
hipError_t launch_reduce(const double *lv, const double *comb, double *ab, double scale,
                         int64_t npad, int nc0, int nc1, int64_t ncmax, hipStream_t st);

// Batched launch_reduce: lv_off / ab_off are byte offsets from `base`; the
// grid of one problem is (ceil(npad / 256), 2 ncmax), flattened as for
// BatchSweep; ncmax_max bounds every problem's ncmax (LDS size).
struct BatchReduce {
  int64_t lv_off, ab_off;
  const double *comb;
  double scale;
  int64_t npad, ncmax;
  int nc0, nc1;
  int wg_start, nbx;
};
hipError_t launch_reduce_batch(const BatchReduce *d, const int *wg_prob, int nwg, int64_t ncmax_max,
                               char *base, hipStream_t st);

// Y_perm[r][col] = x[r][col] + carries (final pass, non-transposed; x of
// storage type T).
// mode 0: write Y in the parity-blocked layout (npad x npad, ld npad);
// mode 1: write the natural-order n x n array, entry (i,j) times
//         sinv_i * sinv_j when `sinv` is non-null;
// mode 2: add Y into the parity-blocked FP64 array `out`.
template <typename T>
hipError_t launch_finalize(const T *x, const double *ab, const double *tab, double *out, int mode,
                           const double *sinv, int64_t n, int64_t npad, int64_t mp0,
                           int64_t mstride, int64_t ncmax, hipStream_t st);

// Residual of the symmetric Sylvester equation in the parity-blocked layout,
// r = G - (A~ Y + Y A~) (Y null: r = G), in FP64, stored in float as r and
// r^T.  A~ acts along each parity block as a tridiagonal stencil with
// diagonal dv[] and coupling ev[] (ev[k] couples positions k and k+1).
hipError_t launch_residual(const double *G, const double *Y, const double *dv, const double *ev,
                           float *r, float *rT, int64_t npad, hipStream_t st);

// natural n x n (ld n) -> parity-blocked npad x npad (zero padding); with
// `sinv` non-null, entry (i, j) is multiplied by sinv[i] * sinv[j].
hipError_t launch_permute_in(const double *src, double *dst, int64_t n, int64_t npad, int64_t mp0,
                             hipStream_t st, const double *sinv = nullptr);

// parity-blocked npad x npad -> natural n x n, entry (i, j) times
// sinv[i] * sinv[j] when sinv is non-null.
hipError_t launch_permute_out(const double *src, double *dst, int64_t n, int64_t npad, int64_t mp0,
                              const double *sinv, hipStream_t st);

hipError_t launch_transpose(const double *src, double *dst, int64_t npad, hipStream_t st);
hipError_t launch_fill(double *dst, int64_t count, double v, hipStream_t st);

// FP64 GEMM on MFMA, up to 4 independent problems per launch:
//   C(i,j) = sum_k A(i,k) B(k,j),  A(i,k) = A[i*sai + k], B(k,j) = B[k*sbk + j],
//   C(i,j) at C[i*sci + j*scj]  (sak and sbj must be 1; K a multiple of 16;
//   A, B 16-byte aligned with even row strides).
// Triangular structure: when triA, A(i,k) = 0 for k < i + offA; when triB,
// B(k,j) = 0 for k < j + offB; k-tiles below the first nonzero are skipped.
struct GemmProb {
  const double *A;
  const double *B;
  double *C;
  int64_t M, N, K;
  int64_t sai, sak, sbk, sbj, sci, scj;
  int triA, offA, triB, offB;
  // upper bounds: when triAu, A(i,k) = 0 for k > i + offAu; when triBu,
  // B(k,j) = 0 for k > j + offBu; k-tiles above the last nonzero are skipped.
  int triAu, offAu, triBu, offBu;
};
hipError_t launch_gemm(const GemmProb *probs, int count, hipStream_t st);

// The launcher's operand requirements (also for table-driven problems, with
// offsets in place of pointers) and the tile count of one problem (ntx: its
// column tiles).
bool gemm_operands_ok(const GemmProb &q);
int gemm_tiles(const GemmProb &q, int *ntx);

// Table-driven GEMM over many problems in one launch.  Each pointer of a
// descriptor's GemmProb is absolute (base id 0), a byte offset from `ws`
// (1) or from `out` (2).  Workgroup g computes tile (local % ntx, local /
// ntx), local = g - tile_start, of problem tile_prob[g].
struct GemmDesc {
  GemmProb p;
  int abase, bbase, cbase;
  int tile_start, ntx;
};
hipError_t launch_gemm_table(const GemmDesc *d, const int *tile_prob, int ntiles, char *ws,
                             char *out, hipStream_t st);

}  // namespace fps
