// Launch interfaces of the gfx950 kernels of the spectral Poisson solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "planner.hpp"

namespace fps {

// One ADI half-sweep.  Chains run down the storage rows of a parity-blocked
// array (npad rows = chain positions of both parities, row stride ld), one
// chain per storage column (ncols of them); nbatch such arrays (e.g. the
// z-slices of a cube) are swept together, batch b at offset b * bstride.
//   input  v = in_scale * in + (carry correction of the producing pass)
//   rhs    r = v + sg * g (g non-null, og == 0) or v; with `pre` non-null, r is
//          first multiplied along the chain by the tridiagonal stencil with
//          diagonal pre[row] and coupling pre[npad + row] (rows row, row + 1)
//   solve  x = T^-1 r along each chain (per parity), T the pass's
//          tridiagonal (tables)
//   output out_mode 0: v + og * g - sigma x stored transposed (requires
//          ncols == ld == npad; the next pass then solves along the other
//          index); 1: x in place orientation; 2: v + og * g - sigma x in place
//          orientation; 3: x stored transposed (as mode 0).  Chunk-level
//          carries are not applied by the
//          producer: it leaves its chunk boundary values in `lv`;
//          launch_reduce turns them into carries, which the consumer (the
//          next sweep, or a finalize kernel) folds in.
// A g array enters either the right-hand side (sg, og == 0) or, on stencil
// passes only, the output base (og, sg == 0).
struct SweepArgs {
  const void *in;          // [npad rows][ld], storage type in_f32
  double in_scale;
  const double *ab_prev;   // producer's chunk carries [2][ncmax][npad][2] (producer chains = npad), or null
  const double *tab_prev;  // producer's per-position tables (its shift) [2][kNTab][mstride]
  // Carries formed in the sweep itself (ctab_prev non-null; chains of at
  // most two chunks per parity, ncmax <= 2): from the producer's chunk
  // boundary values lv_prev (its lv, [ncmax][2][2][npad]) and chunk tables
  // ctab_prev ([2][kNCTab][ncmax]), times carry_scale (the scale launch_reduce
  // would apply); ab_prev is then unused.
  const double *lv_prev;
  const double *ctab_prev;
  double carry_scale;
  const void *g;           // G term, same layout as `in`, or nullptr
  double sg, og;
  const double *tab;       // this pass's tables [2][kNTab][mstride]
  const double *l1;        // this pass's segment-carry combinations [2][ncmax][kL1]
  double sigma;
  void *out;               // storage type out_f32
  double *lv;              // chunk boundary values [ncmax][2][2][ncols]
  const double *pre;       // stencil [2][npad] or nullptr (float64 storage only)
  double pre_shift;        // added to the stencil's diagonal
  int out_mode;
  int64_t npad, mp0, mp1, mstride, ncmax;
  int64_t ncols, ld;       // chains, row stride (elements)
  int nbatch;              // arrays swept together (>= 1)
  int64_t bstride;         // elements between arrays (in, g, out)
  int64_t lvb, abb;        // doubles between the arrays' lv / ab_prev blocks
  int nc0, nc1;
  // Storage types (0: double, 1: float; arithmetic is double throughout).
  // Supported: without g, in/out = d/d, f/d, f/f; with g, in/g/out =
  // d/d/d, d/f/d, f/f/d, f/f/f.  Stencil passes: d/d or f/f without g,
  // d/d/d or f/f/f with g in the right-hand side, d/d/d with g in the
  // output base.
  int in_f32, g_f32, out_f32;
  // Single launches: the chain blocks (64 chains) blk0 .. blk1-1 and chunk
  // rows (parity-0 chunks first) chk0 .. chk1-1 only; blk1 = 0 / chk1 = 0
  // take all of them.  Batched launches take all.
  int blk0, blk1, chk0, chk1;
};

// With ev0 / ev1 non-null the launch records the dispatch's own start and
// end timestamps in them (no separate event packets).
hipError_t launch_sweep(const SweepArgs &a, hipStream_t st, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);

// Row-chain half-sweep: the same pass along the storage rows of `in`
// (chains = rows, positions = columns, ncols = npad chains), stored in the
// same layout (out_mode 1: x, 2: v - sigma x); no g term or stencil, single
// arrays; in/out storage d/d, f/d or f/f.  The producer's carries fold in
// as in launch_sweep with the producer's chains along the columns; its
// chunk boundary values go to lv ([ncmax][2][2][npad], chains = rows).
// Equals launch_sweep on the transposed arrays bit for bit.
hipError_t launch_sweep_rows(const SweepArgs &a, hipStream_t st, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr);

// Batched sweeps over several independent problems in one launch.  The
// workspace pointers of each descriptor's SweepArgs (in, g, out, lv,
// ab_prev) hold byte offsets from `base`; tab, tab_prev, l1 and pre are
// device pointers; ab_prev is used iff tab_prev is non-null.  With a stencil
// (`types.pre` non-null) every descriptor must carry one.  Workgroup g runs
// block (local % nbx, local / nbx), local = g - wg_start, of problem
// wg_prob[g].  Storage types and the presence of g come from `types` /
// `with_g` and must be those of every descriptor.
struct BatchSweep {
  SweepArgs a;
  int wg_start, nbx;
};
// wg_base: the launch runs workgroups wg_base .. wg_base + nwg - 1 of the map.
hipError_t launch_sweep_batch(const SweepArgs &types, bool with_g, const BatchSweep *d,
                              const int *wg_prob, int nwg, char *base, hipStream_t st,
                              int wg_base = 0, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// LDS-resident slice ADI of the z-eigenbasis cube (zeig_lds.hip): for
// every sorted slice k (slice[k] its storage slice, J[k] its steps, 0 for the
// inactive slices, whose Y^ is zeroed), the J[k] steps of the batched slice
// sweeps' pass form (x solve with tables tab0[k] + 2j, y solve with tables
// tab0[k] + 2j + 1 and the stencil pre = A~ + mu[k], the identity at the last
// step; sigmas sig[sig0[k] + 2j], sig[sig0[k] + 2j + 1]) on G^ (npad^3,
// [z][y][x]), writing Y^ = -(the final y solve) for all four parity blocks of
// the slice.  Needs parity blocks of at most 128 (zeig_lds_fits).  The chains are solved in chunks of kZeigLdsChunk
// positions with the chunk multipliers tab32 ([table][2][BF2, Bk2][mstride])
// and ctab32 ([table][2][F2last, BF2first, Bk2first][mstride /
// kZeigLdsChunk]) of fps::build_chunk_tables.
constexpr int kZeigLdsChunk = 16;
//
// The nested cube's inner ADI (`nested`) runs the same kernel with the
// stencil pre = A~ in both solves (the last y solve keeps it), mu = 0, both
// solves of step j on table tab0_all + j, every slice k in storage slice k
// with J_all steps and the sigmas sig[2j], sig[2j + 1], writing +(the final
// y solve).  Null per-slice arrays take these uniform values (slice k, mu 0,
// sig0 0); tab0_all / J_all >= 0 replace tab0[] / J[].
struct ZeigLdsArgs {
  const double *G;
  double *Y;
  const double *tab, *tab32, *ctab32, *pre, *mu, *sig;
  const int *slice, *J, *tab0, *sig0;
  int64_t npad, mp0, mstride, ncmax;
  int m0, m1;
  int tab0_all = -1, J_all = -1;
  // nested: Y receives cy x + cr G + cb B instead of x (B null: cy x)
  const double *B = nullptr;
  double cy = 1.0, cr = 0.0, cb = 0.0;
};
bool zeig_lds_fits(int64_t m0, int64_t m1);
hipError_t launch_zeig_lds(const ZeigLdsArgs &a, int nslices, hipStream_t st,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool nested = false);

// Batched row-chain sweeps (launch_sweep_rows per problem): every
// descriptor is a single array whose chains are its storage rows, with
// out_mode 0 (v - sigma x) or 3 (x), stored in the input's layout; no g term
// or stencil; in/out storage d/d, f/d or f/f from `types`.  Workgroup g runs
// chain block local % nbx and chunk row local / nbx of problem wg_prob[g].
hipError_t launch_sweep_batch_rows(const SweepArgs &types, const BatchSweep *d, const int *wg_prob,
                                   int nwg, char *base, hipStream_t st, int wg_base = 0,
                                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Chunk carries: for every chain, the forward and backward carry into each
// chunk, scaled by `scale`, into ab [2][ncmax][nchains][2] (ctab: the
// per-chunk coefficients [2][kNCTab][ncmax] of the producing pass's shift);
// nbatch blocks of lv / ab at strides lvb / abb.
// Only the chains r_lo .. r_hi-1 (r_hi < 0: all) of the parities s_lo ..
// s_hi-1 are resolved.
hipError_t launch_reduce(const double *lv, const double *ctab, double *ab, double scale,
                         int64_t nchains, int nc0, int nc1, int64_t ncmax, hipStream_t st,
                         int nbatch = 1, int64_t lvb = 0, int64_t abb = 0, int64_t r_lo = 0,
                         int64_t r_hi = -1, int s_lo = 0, int s_hi = 2);

// Shape of the chunk-carry kernels for chains of up to ncmax chunks: each
// chain on a segment of 2 to 16 lanes (the least power of two that holds
// min(ncmax, 16) lanes), and 256 / lanes chains per workgroup (256 threads).
constexpr int kReduceThreads = 256;
constexpr int kReduceMaxLanes = 16;
inline int reduce_lanes(int64_t ncmax) {
  int l = 2;
  while (l < kReduceMaxLanes && l < ncmax) l <<= 1;
  return l;
}
inline int reduce_chains(int64_t ncmax) { return kReduceThreads / reduce_lanes(ncmax); }

// Batched launch_reduce: lv_off / ab_off are byte offsets from `base`; the
// workgroups of one problem are (chain block b, parity s) -> local index
// s * nbx + b with nbx = ceil(npad / reduce_chains(ncmax_max)), flattened as for
// BatchSweep; ncmax_max bounds every problem's ncmax (lanes per chain).
struct BatchReduce {
  int64_t lv_off, ab_off;
  const double *ctab;
  double scale;
  int64_t npad, ncmax;
  int nc0, nc1;
  int wg_start, nbx;
};
// wg_base: the launch runs workgroups wg_base .. wg_base + nwg - 1 of the map.
hipError_t launch_reduce_batch(const BatchReduce *d, const int *wg_prob, int nwg, int64_t ncmax_max,
                               char *base, hipStream_t st, int wg_base = 0);

// Y_perm[r][col] = x[r][col] + carries (final pass, non-transposed; x of
// storage type T).
// mode 0: write Y in the parity-blocked layout (npad x npad, ld npad);
// mode 1: write the natural-order n x n array, entry (i,j) times
//         sinv_i * sinv_j when `sinv` is non-null;
// mode 2: add Y into the parity-blocked FP64 array `out`.
// Only the parity-blocked rows r0 .. r1-1 (r1 < 0: all) are finalized.
template <typename T>
hipError_t launch_finalize(const T *x, const double *ab, const double *tab, double *out, int mode,
                           const double *sinv, int64_t n, int64_t npad, int64_t mp0,
                           int64_t mstride, int64_t ncmax, hipStream_t st, int64_t r0 = 0,
                           int64_t r1 = -1);

// Residual of the symmetric Sylvester equation in the parity-blocked layout,
// r = G - (A~ Y + Y A~) (Y null: r = G), in FP64, stored in float as r and,
// with rT non-null, r^T.  A~ acts along each parity block as a tridiagonal stencil with
// diagonal dv[] and coupling ev[] (ev[k] couples positions k and k+1).
// For a rectangle the operator is ax A~ Y + ay Y A~ (ax = sx2, ay = sy2).
// Only the rows r0 .. r1-1 (multiples of 64; r1 < 0: all) are formed (rT
// only with all rows); rows across a zero coupling are not read.
hipError_t launch_residual(const double *G, const double *Y, const double *dv, const double *ev,
                           float *r, float *rT, int64_t npad, hipStream_t st, double ax = 1.0,
                           double ay = 1.0, int64_t r0 = 0, int64_t r1 = -1);

// natural n x n (ld n) -> parity-blocked npad x npad (zero padding); with
// `sinv` non-null, entry (i, j) is multiplied by sinv[i] * sinv[j].
hipError_t launch_permute_in(const double *src, double *dst, int64_t n, int64_t npad, int64_t mp0,
                             hipStream_t st, const double *sinv = nullptr);

// parity-blocked npad x npad -> natural n x n, entry (i, j) times
// sinv[i] * sinv[j] when sinv is non-null.
hipError_t launch_permute_out(const double *src, double *dst, int64_t n, int64_t npad, int64_t mp0,
                              const double *sinv, hipStream_t st);

// One problem of a batched element-wise launch (launch_permute_in,
// launch_residual or launch_finalize for many problems at once, each
// workgroup doing what the single-problem launch's workgroup does).
// Workgroups wg_start .. of the launch belong to this problem, nbx per row
// of its own grid (permute-in, finalize: ceil(npad / 256) per row, npad
// rows; residual: npad / 64 tiles per row of tiles).  src / dst
// are byte offsets from the base named by sbase / dbase (0: absolute, 1:
// workspace, 2: the input F); ab is a workspace offset, tab and ev device
// pointers.  The residual takes G at src, Y at ab, r at dst, the stencil's
// diagonal at tab and its coupling at ev.
struct ElemDesc {
  int64_t src, dst, ab;
  const double *tab, *ev;
  int64_t n, npad, mp0, mstride, ncmax;
  int sbase, dbase;
  int wg_start, nbx;
};
// F of every problem into its parity-blocked layout (no sinv).
hipError_t launch_permute_in_batch(const ElemDesc *d, const int *wg_prob, int nwg, const double *in,
                                   char *ws, hipStream_t st);
// launch_residual (ax = ay = 1) for every problem; with_y false: r = G.
hipError_t launch_residual_batch(const ElemDesc *d, const int *wg_prob, int nwg, bool with_y,
                                 char *ws, hipStream_t st);
// launch_finalize with mode 0 or 2 (no sinv), the input x in float when
// x_f32 is set, else in double.
hipError_t launch_finalize_batch(const ElemDesc *d, const int *wg_prob, int nwg, int mode, char *ws,
                                 hipStream_t st, int x_f32 = 0);

// Cube (npad^3 arrays [z][y][x], every axis parity-blocked):
// natural n^3 -> parity-blocked npad^3 (zero padding).
hipError_t launch_permute3_in(const double *src, double *dst, int64_t n, int64_t npad, int64_t mp0,
                              hipStream_t st);
// parity-blocked (row length ld, parity-1 blocks at mb0 on every axis) ->
// natural N^3, times sinv_i sinv_j sinv_k when sinv is non-null.
hipError_t launch_permute3_out(const double *src, double *dst, int64_t N, int64_t ld, int64_t mb0,
                               const double *sinv, hipStream_t st);
// After a z-fiber sweep: R = x + chunk carries (ab over the npad^2 (y, x)
// chains, tab of the sweep's shift), stored as R[z][y][x] and, unless RT is
// null, R^T[z][x][y].
hipError_t launch_cube_zfinal(const double *x, const double *ab, const double *tab, double *R,
                              double *RT, int64_t npad, int64_t mp0, int64_t mstride,
                              int64_t ncmax, hipStream_t st);
// Per-slice finalization with a table per slice: v = scale (x[z] + chunk
// carries of slice z) when tabs[z] is non-null, else 0; out[z] = v, or
// out[z] += v with `add` (x of storage type T).
template <typename T>
hipError_t launch_slice_final(const T *x, const double *ab, const double *const *tabs, double *out,
                              double scale, int add, int64_t npad, int64_t mp0, int64_t mstride,
                              int64_t ncmax, hipStream_t st);
// z-eigenbasis cube, refinement: the negated residual of every slice
// equation, q_z = G_z + A~ Y_z A~ + mu[z] (A~ Y_z + Y_z A~) (Y null: q = G),
// FP64 arithmetic, stored in float; dv / ev the A~ stencil of
// launch_residual; nslices arrays of npad x npad at stride npad^2.
hipError_t launch_zeig_residual(const double *G, const double *Y, const double *dv, const double *ev,
                                const double *mu, float *q, int64_t npad, int64_t nslices,
                                hipStream_t st);
// After a row solve of every slice that left x in place (float, chunk
// carries pending in ab at the per-slice stride 2 ncmax npad 2, tables tab
// shared by the slices): v = x + carries stored in float both as outT (x's
// orientation) and out (transposed).
hipError_t launch_slice_xfinal(const float *x, const double *ab, const double *tab, float *outT,
                               float *out, int64_t npad, int64_t mp0, int64_t mstride,
                               int64_t ncmax, int64_t nslices, hipStream_t st);
// After the last per-slice sweep (chains = x, positions = y, ab per slice):
// out = cy (x + chunk carries) + cr R + cb B; ab null: x is complete.
hipError_t launch_cube_ifinal(const double *x, const double *ab, const double *tab,
                              const double *R, const double *B, double *out, double cy, double cr,
                              double cb, int64_t npad, int64_t mp0, int64_t mstride, int64_t ncmax,
                              hipStream_t st);
hipError_t launch_fill(double *dst, int64_t count, double v, hipStream_t st);

// Nonhomogeneous Dirichlet data (Sec. 6.1), traces bc = [L; R; B; T], each
// n + 2 Chebyshev coefficients in the mapped variable (L, R in t; B, T in s).
// Constants of the lift: sinv[i] = 1/sqrt((i+1)(i+2)) and the C~
// coefficients am / ap of (1 - t)/2 and (1 + t)/2 at degrees 0 and 1.
struct BcLiftConst {
  double sinv[2], am[2], ap[2];
};
// G (parity-blocked, row stride npad) -= S^-1 C~(Lap u_bc) S^-1, touching
// rows 0, 1 and columns 0, 1 only.  Ms0 / Ms1: the lift map S^-1 C~(T_k'')
// by parity (m_s x mo_s, row-major, build_lift_map).  scratch: [4][npad] +
// [8] doubles; its last 8 entries keep the traces' values at -1 and +1 for
// launch_bc_lift_out.
hipError_t launch_bc_lift_rhs(const double *bc, const double *Ms0, const double *Ms1, double *G,
                              double *scratch, const Layout &L, double sx2, double sy2,
                              const BcLiftConst &k, hipStream_t st);
// Cylinder: F [mode][part][n][n] -> X0 [slot][part][r][z] parity-blocked
// (slot -> mode through slot_idx), zero padded to npad = 2 mp per axis.
hipError_t launch_cyl_permute_in(const double *F, double *X0, const int *slot_idx, int64_t n,
                                 int64_t nt, int64_t mp, hipStream_t st);
// Cylinder: the right-hand sides that share one |k| (modes k and -k, real
// and imaginary parts): up to kCylRhs (slot * 2 + part) rows of X0 / X1,
// unused entries -1; rp / wp the row parities of the right-hand side and of
// the solution.
constexpr int kCylRhs = 4;
struct CylSolveGroup {
  int sp[kCylRhs];
  int kabs, rp, wp;
};
// Cylinder: the banded r-solves of every (|k| group, z column) with the
// plan's LU factors (see cylinder.cpp), one thread applying them to all the
// group's right-hand sides; X0 holds the right-hand sides (rows of parity
// rp, overwritten), X1 receives yhat (rows of parity wp).
hipError_t launch_cyl_solve(double *X0, double *X1, const double *fac, const CylSolveGroup *grp,
                            int ngroups, int64_t m, int64_t mp, hipStream_t st);
// Cylinder: the thin edges of the r output map of one (slot, part, z parity)
// problem U_blk = Pr X0_blk (Pr ro x mp row-major, PrT its transpose, X0_blk
// rows of stride mobar in the workspace at byte offset b_off, U_blk at
// element offset c_off with row stride ldc and column stride 2): the rows
// ro_main.. (every column) and the columns mo_main.. of the rows above
// ro_main, at most 8 of each, mp <= 256.  One workgroup per problem.
struct CylEdge {
  const double *Pr, *PrT;
  int64_t b_off, c_off;
};
hipError_t launch_cyl_redge(const CylEdge *d, int nprob, char *ws, double *U, int64_t mp,
                            int64_t ro, int64_t ro_main, int64_t mo, int64_t mo_main,
                            int64_t mobar, int64_t ldc, hipStream_t st);

// U ((n+2) x (n+2) Chebyshev, natural order) += coefficients of u_bc.
hipError_t launch_bc_lift_out(double *U, const double *bc, const double *scratch, int64_t n,
                              int64_t npad, hipStream_t st);

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
// ntx) of problem tile_map[2g], local = tile_map[2g + 1].
struct GemmDesc {
  GemmProb p;
  int abase, bbase, cbase;
  int tile_start;  // first tile of this problem in table order (host bookkeeping)
  int ntx;
};
hipError_t launch_gemm_table(const GemmDesc *d, const int *tile_map, int ntiles, char *ws,
                             char *out, hipStream_t st);
// Host: the tile map of a table, (problem, local tile) pairs for every tile
// of every problem, longest k-range (after the triangular skips) first.
std::vector<int> gemm_table_map(const std::vector<GemmDesc> &tab);
// Output tile of the MFMA GEMMs (rows and columns).
constexpr int kGemmTile = 128;
// The columns tn.. (a thin edge past whole tiles, whose MFMA tiles would be
// almost empty) of every row of each table problem, in plain FP64 FMAs:
// one wavefront per row with coalesced loads along k and a fixed-order sum
// across the wavefront; problems without triangular structure only; nblk
// workgroups of 4 wavefronts per problem, interleaved (workgroup b serves
// problem b % nprob), 4 rows per wavefront iteration (8 on the vector path
// for k-contiguous, 16-byte aligned rows).
hipError_t launch_gemm_edge_cols(const GemmDesc *d, int nprob, int64_t tn, int nblk, char *ws,
                                 char *out, hipStream_t st);
// Leading extent of a dimension split off a thin edge: x less its last
// partial tile when that tile holds at most 8 rows or columns, else x.
inline int64_t gemm_main_extent(int64_t x) {
  const int64_t r = x % kGemmTile;
  return x > kGemmTile && r != 0 && r <= 8 ? x - r : x;
}

}  // namespace fps
