// C ABI of the spectral Poisson solver (declared in include/fps.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "solver.hpp"

namespace fps {
namespace detail {

namespace {
thread_local std::string g_last_error;
}

fps_status fail(fps_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

const char *last_error() { return g_last_error.c_str(); }

bool valid_plan(const fps_plan *p) { return p != nullptr && p->magic == kMagic; }

void spectrum_tight(int64_t n, double *a, double *b) {
  long double lmin, lmax;
  fps::atilde_extremes(n, &lmin, &lmax);
  constexpr long double kMargin = 1e-6L;  // relative widening (bisection and rounding)
  *a = (double)(lmin * (1.0L + kMargin));
  *b = (double)(lmax * (1.0L - kMargin));
}

int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

hipError_t timed_sweep(fps_plan *pl, const fps::SweepArgs &a, hipStream_t st, bool rows) {
  const auto launch = rows ? fps::launch_sweep_rows : fps::launch_sweep;
  const bool t = pl->ev_used * 2 + 1 < (int64_t)pl->ev.size();
  if (!t) return launch(a, st, nullptr, nullptr);
  const hipError_t e = launch(a, st, pl->ev[2 * pl->ev_used], pl->ev[2 * pl->ev_used + 1]);
  if (e == hipSuccess) ++pl->ev_used;
  return e;
}

void release_events(fps_plan *pl) {
  for (hipEvent_t e : pl->ev) (void)hipEventDestroy(e);
  pl->ev.clear();
  pl->ev_used = 0;
}

// Whether the 2-D plan's solves run their two row-parity blocks on two
// streams: the plan has its side stream (chains of more than two chunks and
// both blocks non-empty), and sweep timing (every launch on the caller's
// stream) is off.
bool row_split(const fps_plan *pl) {
  return pl->zside != nullptr && pl->dim == 2 && pl->L.ncmax > 2 && pl->L.m[1] > 0 &&
         pl->ev.empty();
}

// Runs body(r0, r1, c0, c1, s, stream) -- a part of a solve restricted to
// the storage rows r0 .. r1-1 of row-parity block s (chunk rows c0 .. c1-1
// of that block), returning a hipError_t -- once on the whole array on st,
// or, with row_split(pl), for block 1 on the plan's side stream and block 0
// on st.  One solve at a time forks onto the side stream (its event record
// and wait must not interleave with another host thread's); the join is
// enqueued whatever the parts returned, so the side stream (or a graph being
// captured) is never left forked.
template <typename Body>
fps_status for_row_blocks(fps_plan *pl, hipStream_t st, Body body) {
  const fps::Layout &L = pl->L;
  const int nc0 = (int)L.nc[0], nc1 = (int)L.nc[1];
  if (!row_split(pl)) {
    FPS_HIP(body(0, L.npad, 0, nc0 + nc1, 0, st));
    return FPS_OK;
  }
  std::lock_guard<std::mutex> lk(pl->zlock);
  FPS_HIP(hipEventRecord(pl->zfork, st));
  FPS_HIP(hipStreamWaitEvent(pl->zside, pl->zfork, 0));
  const hipError_t e1 = body(L.mp[0], L.npad, nc0, nc0 + nc1, 1, pl->zside);
  const hipError_t e2 = e1 == hipSuccess ? body(0, L.mp[0], 0, nc0, 0, st) : hipSuccess;
  const hipError_t e3 = hipEventRecord(pl->zjoin, pl->zside);
  const hipError_t e4 = e3 == hipSuccess ? hipStreamWaitEvent(st, pl->zjoin, 0) : e3;
  FPS_HIP(e1);
  FPS_HIP(e2);
  FPS_HIP(e3);
  FPS_HIP(e4);
  return FPS_OK;
}

// The J steps of Algorithm 2 (see run_adi) on the storage rows r0 .. r1-1
// of one row-parity block s (chunk rows c0 .. c1-1 of the second
// half-steps), or with r0 = 0, r1 = npad on the whole array, enqueued on s2.
// A~ is block diagonal in the parity-blocked layout, so the rows of one
// parity block iterate independently of the other block's: the first
// half-step solves along those rows (chain blocks r0 / 64 ..), the second
// along every column but only over those rows, and each half-step's carries
// are those of its own chains and positions.
hipError_t adi_part(fps_plan *pl, const fps::ShiftSet &sh, int base, const void *Gterm, int g_f32,
                    int f32, void *O0, void *O1, char *ws, int64_t r0, int64_t r1, int c0, int c1,
                    int s, hipStream_t s2) {
  const fps::Layout &L = pl->L;
  const int J = sh.J;
  const std::vector<double> &p = sh.p, &q = sh.q;
  double *lv = (double *)(ws + pl->off_lv), *lv2 = (double *)(ws + pl->off_lv2);
  double *ab = (double *)(ws + pl->off_ab), *ab2 = (double *)(ws + pl->off_ab2);
  const int nc0 = (int)L.nc[0], nc1 = (int)L.nc[1];
  // Chains of at most two chunks: each sweep forms its producer's carries
  // itself from the boundary values (first half-steps write lv, second ones
  // lv2), and only the last half-step's carries are launched (for the final
  // pass).  Longer chains: a carry launch after every half-step (first
  // half-steps' carries into ab2, second ones' into ab).
  const bool fused = L.ncmax <= 2;
  fps::SweepArgs A0{};
  A0.npad = L.npad;
  A0.ncols = L.npad;
  A0.ld = L.npad;
  A0.nbatch = 1;
  A0.mp0 = L.mp[0];
  A0.mp1 = L.mp[1];
  A0.mstride = L.mstride;
  A0.ncmax = L.ncmax;
  A0.nc0 = nc0;
  A0.nc1 = nc1;
  const bool whole = r0 == 0 && r1 == L.npad;
  double sigma_prev = 0.0;
  for (int j = 0; j < J; ++j) {
    const double s1 = pl->rect ? p[j] - q[j] : 2.0 * p[j];
    fps::SweepArgs A = A0;
    if (!whole) {
      A.blk0 = (int)(r0 / 64);
      A.blk1 = (int)(r1 / 64);
    }
    A.in = j == 0 ? Gterm : (const void *)O1;
    A.in_f32 = j == 0 ? g_f32 : f32;
    A.in_scale = j == 0 ? -1.0 : 1.0;
    A.ab_prev = j == 0 ? nullptr : ab;
    A.tab_prev = j == 0 ? nullptr : pl->tab_dev(pl->tab2(base + j - 1));
    A.tab = pl->tab_dev(pl->tab1(base + j));
    A.l1 = pl->l1_dev(pl->tab1(base + j));
    A.sigma = s1;
    A.out = O0;
    A.out_f32 = f32;
    A.out_mode = 2;
    if (fused && j > 0) {
      A.ab_prev = nullptr;
      A.lv_prev = lv2;
      A.ctab_prev = pl->ctab_dev(pl->tab2(base + j - 1));
      A.carry_scale = -sigma_prev;
    }
    A.lv = lv;
    hipError_t e = timed_sweep(pl, A, s2, true);
    if (e == hipSuccess && !fused)
      e = fps::launch_reduce(lv, pl->ctab_dev(pl->tab1(base + j)), ab2, -A.sigma, L.npad, nc0,
                             nc1, L.ncmax, s2, 1, 0, 0, r0, r1, 0, 2);
    if (e != hipSuccess) return e;
    fps::SweepArgs B = A0;
    if (!whole) {
      B.chk0 = c0;
      B.chk1 = c1;
    }
    const bool last = j == J - 1;
    B.in = O0;
    B.in_f32 = f32;
    B.in_scale = 1.0;
    B.ab_prev = ab2;
    B.tab_prev = A.tab;
    if (fused) {
      B.ab_prev = nullptr;
      B.lv_prev = lv;
      B.ctab_prev = pl->ctab_dev(pl->tab1(base + j));
      B.carry_scale = -A.sigma;
    }
    B.lv = lv2;
    B.g = Gterm;
    B.g_f32 = g_f32;
    B.sg = 1.0;
    B.tab = pl->tab_dev(pl->tab2(base + j));
    B.l1 = pl->l1_dev(pl->tab2(base + j));
    B.sigma = last ? 0.0 : (pl->rect ? p[j + 1] - q[j] : p[j] + p[j + 1]);
    B.out = O1;
    B.out_f32 = f32;
    B.out_mode = last ? 1 : 2;
    e = timed_sweep(pl, B, s2);
    if (e == hipSuccess && (!fused || last))
      e = fps::launch_reduce(lv2, pl->ctab_dev(pl->tab2(base + j)), ab, last ? 1.0 : -B.sigma,
                             L.npad, nc0, nc1, L.ncmax, s2, 1, 0, 0, 0, L.npad,
                             whole ? 0 : s, whole ? 2 : s + 1);
    if (e != hipSuccess) return e;
    sigma_prev = B.sigma;
  }
  return hipSuccess;
}

// Runs the 2J half-sweeps of Algorithm 2 with the shifts `sh`, whose step j
// uses the plan's tables of step base + j.  `Gterm` is the right-hand side G
// (parity-blocked, npad x npad) of storage type g_f32; O0, O1 are the
// ping-pong arrays (room for npad^2 doubles each), in G's layout.  With f32 set every step stores its outputs in float (refinement
// rounds, including the final chunk-local solution: a later round corrects
// its rounding, and the last round's correction is small), else in double.
// Leaves the final chunk-local solution in O1 and its chunk carries in ab,
// to finalize with the tables of the last second half-step
// (pl->tab2(base + J - 1)).
//
// Every array keeps one layout (that of G): half-step 1 solves along its
// storage rows (launch_sweep_rows), half-step 2 along its storage columns
// (launch_sweep), and both store their outputs in place of their inputs'
// layout.
// Algorithm 2 for A Y - Y B = G with T1_j = -(B - p_j) (first half-step,
// along the columns of Y) and T2_j = A - q_j (second half-step, along the
// rows).  Half-step 1: right-hand side R_j = (A - p_j) Y_j - G, solve
// Y_{j+1/2} T1_j = R_j, output V_j - G = R_j - (p_j - q_j) Y_{j+1/2}
// (V_j = G - Y_{j+1/2}(B - q_j) and Y_{j+1/2}(B - q_j) = -R_j +
// (p_j - q_j) Y_{j+1/2}).  Half-step 2: right-hand side V_j = (V_j - G) + G,
// solve T2_j Y_{j+1} = V_j, output R_{j+1} = (V_j - G) - (p_{j+1} - q_j)
// Y_{j+1}.  So only half-step 2 reads G, and R_0 = -G.  For the square
// (q_j = -p_j, T1_j = T2_j = A~ + p_j) the coefficients are 2 p_j and
// p_j + p_{j+1}.  After every half-step the chunk carries are resolved,
// and the next half-step folds them in.
fps_status run_adi(fps_plan *pl, const fps::ShiftSet &sh, int base, const void *Gterm, int g_f32,
                   int f32, void *O0, void *O1, char *ws, hipStream_t st) {
  return for_row_blocks(pl, st, [&](int64_t r0, int64_t r1, int c0, int c1, int s, hipStream_t s2) {
    return adi_part(pl, sh, base, Gterm, g_f32, f32, O0, O1, ws, r0, r1, c0, c1, s, s2);
  });
}

// The symmetric-form solution Y (parity-blocked FP64, npad x npad) of
// A~ Y + Y A~ = G for G in ws.G, on the rows r0 .. r1-1 of row-parity block
// s (see adi_part; the whole array with r0 = 0, r1 = npad): plain FP64 ADI
// (Y left in G), or iterative refinement whose inner ADIs store their sweep
// arrays in float (Y in the GT region).  A~ is block diagonal, so the
// residual of a row block needs only that block's rows.
hipError_t symmetric_part(fps_plan *pl, char *w, int64_t r0, int64_t r1, int c0, int c1, int s,
                          hipStream_t s2) {
  const fps::Layout &L = pl->L;
  double *G = (double *)(w + pl->off_G);
  double *ab = (double *)(w + pl->off_ab);
  hipError_t e;
  if (pl->prec == FPS_FP64) {
    const int J = pl->shifts.J;
    e = adi_part(pl, pl->shifts, 0, G, 0, 0, w + pl->off_O0, w + pl->off_O1, w, r0, r1, c0, c1, s,
                 s2);
    if (e != hipSuccess) return e;
    return fps::launch_finalize<double>((const double *)(w + pl->off_O1), ab,
                                        pl->tab_dev(pl->tab2(J - 1)), G, 0, nullptr, L.n, L.npad,
                                        L.mp[0], L.mstride, L.ncmax, s2, r0, r1);
  }
  // Refinement: Y <- Y + ADI_k(G - (A~ Y + Y A~)) for the rounds k; the
  // residual is formed in FP64 and stored in float, and the inner sweeps of
  // a float round store their arrays in float.
  double *Y = (double *)(w + pl->off_GT);
  float *r = (float *)(w + pl->off_R);
  for (int k = 0; k < pl->rounds; ++k) {
    const fps::ShiftSet &sh = pl->rsh[(size_t)k];
    const int f32 = pl->rf32[(size_t)k];
    const double *tab = pl->tab_dev(pl->tab2(pl->rbase[(size_t)k] + sh.J - 1));
    void *O0 = w + pl->off_O0, *O1 = w + pl->off_O1;
    e = fps::launch_residual(G, k == 0 ? nullptr : Y, (const double *)pl->d_sdiag.p,
                             (const double *)pl->d_soff.p, r, nullptr, L.npad, s2, pl->sx2,
                             pl->sy2, r0, r1);
    if (e == hipSuccess)
      e = adi_part(pl, sh, pl->rbase[(size_t)k], r, 1, f32, O0, O1, w, r0, r1, c0, c1, s, s2);
    if (e != hipSuccess) return e;
    const int mode = k == 0 ? 0 : 2;
    if (f32)
      e = fps::launch_finalize<float>((const float *)O1, ab, tab, Y, mode, nullptr, L.n, L.npad,
                                      L.mp[0], L.mstride, L.ncmax, s2, r0, r1);
    else
      e = fps::launch_finalize<double>((const double *)O1, ab, tab, Y, mode, nullptr, L.n, L.npad,
                                       L.mp[0], L.mstride, L.ncmax, s2, r0, r1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Y of A~ Y + Y A~ = G for G in ws.G (both row-parity blocks, on two streams
// when the plan splits them).  Returns Y's location.
fps_status solve_symmetric(fps_plan *pl, char *w, hipStream_t st, double **Yout) {
  const fps_status s =
      for_row_blocks(pl, st, [&](int64_t r0, int64_t r1, int c0, int c1, int sp, hipStream_t s2) {
        return symmetric_part(pl, w, r0, r1, c0, c1, sp, s2);
      });
  if (s != FPS_OK) return s;
  *Yout = (double *)(w + (pl->prec == FPS_FP64 ? pl->off_G : pl->off_GT));
  return FPS_OK;
}

fps_status check_solve_args(fps_plan *pl, const void *a, const void *b, void *ws) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (!pl->on_device) return fail(FPS_E_STATE, "plan was created host-only");
  if (!a || !b || !ws) return fail(FPS_E_ARG, "null pointer argument");
  if (((uintptr_t)ws) % 256 != 0) return fail(FPS_E_ARG, "workspace must be 256-byte aligned");
  return FPS_OK;
}

// Input map: G_perm = Rs_s F_st Rs_t^T for the four parity blocks.
int rhs_gemms(const fps_plan *pl, char *ws, fps::GemmProb *g1, fps::GemmProb *g2) {
  const fps::Layout &L = pl->L;
  const int64_t npad = L.npad;
  double *G = (double *)(ws + pl->off_G);
  const double *GT = (const double *)(ws + pl->off_GT);
  double *Tb = (double *)(ws + pl->off_O0);
  int cnt = 0;
  int64_t toff = 0;
  for (int s = 0; s < 2; ++s)
    for (int t = 0; t < 2; ++t) {
      const int64_t ms = L.mp[s], mt = L.mp[t];
      if (ms == 0 || mt == 0) continue;
      double *Tst = Tb + toff;
      toff += ms * mt;
      const double *Fst = GT + (s * L.mp[0]) * npad + t * L.mp[0];
      // T_st = F_st Rs_t^T; B(k, j) = Rs_t[j][k] = 0 for k < j.
      g1[cnt] = fps::GemmProb{Fst, (const double *)pl->d_RsB[t].p, Tst, ms, mt, mt,
                              npad, 1, mt, 1, mt, 1, 0, 0, 1, 0, 0, 0, 0, 0};
      // G_st = Rs_s T_st; A(i, k) = Rs_s[i][k] = 0 for k < i.
      g2[cnt] = fps::GemmProb{(const double *)pl->d_RsA[s].p, Tst,
                              G + (s * L.mp[0]) * npad + t * L.mp[0], ms, mt, ms,
                              ms, 1, mt, 1, npad, 1, 1, 0, 0, 0, 0, 0, 0, 0};
      ++cnt;
    }
  return cnt;
}

// Constants of the Dirichlet lift.  C~_0 = sqrt(3)/2 and C~_1(t) =
// sqrt(5/12) 3t (normalization of Sec. 3.1), so under the weight (1 - t^2)
// <1, C~_0> = 2/sqrt(3) and <t, C~_1> = 2/sqrt(15): (1 -+ t)/2 has C~
// coefficients 1/sqrt(3) and -+1/sqrt(15).
fps::BcLiftConst bc_lift_const() {
  fps::BcLiftConst k;
  k.sinv[0] = 1.0 / std::sqrt(2.0);
  k.sinv[1] = 1.0 / std::sqrt(6.0);
  k.am[0] = k.ap[0] = 1.0 / std::sqrt(3.0);
  k.ap[1] = 1.0 / std::sqrt(15.0);
  k.am[1] = -k.ap[1];
  return k;
}

fps_status rhs_transform(fps_plan *pl, const double *F, char *ws, hipStream_t st, const double *bc) {
  const fps::Layout &L = pl->L;
  // F in the parity-blocked layout (zero padded), staged in the GT region.
  FPS_HIP(fps::launch_permute_in(F, (double *)(ws + pl->off_GT), L.n, L.npad, L.mp[0], st));
  fps::GemmProb g1[4], g2[4];
  const int cnt = rhs_gemms(pl, ws, g1, g2);
  FPS_HIP(fps::launch_gemm(g1, cnt, st));
  FPS_HIP(fps::launch_gemm(g2, cnt, st));
  if (bc)
    FPS_HIP(fps::launch_bc_lift_rhs(bc, (const double *)pl->d_lift[0].p,
                                    (const double *)pl->d_lift[1].p, (double *)(ws + pl->off_G),
                                    (double *)(ws + pl->off_bc), L, pl->sx2, pl->sy2,
                                    bc_lift_const(), st));
  return FPS_OK;
}

int out_gemms(const fps_plan *pl, const double *Y, double *U, char *ws, fps::GemmProb *g1,
              fps::GemmProb *g2) {
  const fps::Layout &L = pl->L;
  const int64_t N = L.n + 2, npad = L.npad;
  // temporaries mp_s x mop_t in the O0 and O1 regions (contiguous, free here)
  double *Tb = (double *)(ws + pl->off_O0);
  int cnt = 0;
  int64_t toff = 0;
  for (int s = 0; s < 2; ++s)
    for (int t = 0; t < 2; ++t) {
      const int64_t ms = L.mp[s], mt = L.mp[t], mot = pl->mop[t];
      if (L.m[s] == 0 || L.m[t] == 0) continue;  // that output block stays zero
      double *Tst = Tb + toff;
      toff += ms * mot;
      // T_st = Y_st P_t^T; B(k, j) = P_t[j][k] = 0 for k < j - 1.
      g1[cnt] = fps::GemmProb{Y + (s * L.mp[0]) * npad + t * L.mp[0], (const double *)pl->d_PB[t].p,
                              Tst, ms, mot, mt, npad, 1, mot, 1, mot, 1, 0, 0, 1, -1, 0, 0, 0, 0};
      // U_st = P_s T_st; A(i, k) = P_s[i][k] = 0 for k < i - 1.
      g2[cnt] = fps::GemmProb{(const double *)pl->d_PA[s].p, Tst, U + s * N + t, L.mo[s], L.mo[t],
                              ms, ms, 1, mot, 1, 2 * N, 2, 1, -1, 0, 0, 0, 0, 0, 0};
      ++cnt;
    }
  return cnt;
}

fps_status out_transform(fps_plan *pl, const double *Y, double *U, char *ws, hipStream_t st) {
  const fps::Layout &L = pl->L;
  const int64_t N = L.n + 2;
  if (L.npad * (pl->mop[0] + pl->mop[1]) * 8 > pl->off_lv - pl->off_O0)
    return fail(FPS_E_STATE, "internal: output temporary exceeds workspace");
  fps::GemmProb g1[4], g2[4];
  const int cnt = out_gemms(pl, Y, U, ws, g1, g2);
  FPS_HIP(fps::launch_fill(U, N * N, 0.0, st));
  FPS_HIP(fps::launch_gemm(g1, cnt, st));
  FPS_HIP(fps::launch_gemm(g2, cnt, st));
  return FPS_OK;
}

// Validates the arguments shared by every plan kind and allocates the plan.
fps_status plan_common(fps_plan **out, int dim, int64_t n, int bc, double tol, int prec,
                       int out_basis, unsigned flags) {
  if (dim != 2 && dim != 3) return fail(FPS_E_ARG, "dim must be 2 or 3");
  if (n < 1) return fail(FPS_E_ARG, "n must be >= 1");
  if (n > 200000) return fail(FPS_E_ARG, "n too large");
  // Square and rectangle plans: chains of up to 8192 positions per parity
  // (128 chunks), the largest the chunk-carry scan keeps in registers.
  if (dim == 2 && n > 16384) return fail(FPS_E_UNSUPPORTED, "square and rectangle plans need n <= 16384");
  if (bc != FPS_BC_DIRICHLET_ZERO) return fail(FPS_E_UNSUPPORTED, "only zero Dirichlet data");
  if (!(tol > 0.0 && tol < 1.0)) return fail(FPS_E_ARG, "tol must lie in (0, 1)");
  if (prec != FPS_FP64 && prec != FPS_FP32_REFINED) return fail(FPS_E_ARG, "bad precision");
  if (out_basis != FPS_OUT_CHEB && out_basis != FPS_OUT_NATIVE) return fail(FPS_E_ARG, "bad out_basis");
  if (flags & ~(FPS_PLAN_HOST_ONLY | FPS_PLAN_TIGHT_SPECTRUM | FPS_PLAN_CUBE_ZEIG |
                FPS_PLAN_DIRICHLET))
    return fail(FPS_E_ARG, "unknown flags");
  if ((flags & FPS_PLAN_DIRICHLET) && dim != 2)
    return fail(FPS_E_UNSUPPORTED, "FPS_PLAN_DIRICHLET applies to square and rectangle plans");
  if ((flags & FPS_PLAN_CUBE_ZEIG) && dim != 3)
    return fail(FPS_E_ARG, "FPS_PLAN_CUBE_ZEIG applies to cube plans only");
  if ((flags & FPS_PLAN_CUBE_ZEIG) && n > 512)
    return fail(FPS_E_UNSUPPORTED, "the z-eigenbasis cube method is limited to n <= 512");
  if (dim == 3 && prec != FPS_FP64 && !(flags & FPS_PLAN_CUBE_ZEIG))
    return fail(FPS_E_UNSUPPORTED,
                "FP32_REFINED cube plans need the z-eigenbasis method (FPS_PLAN_CUBE_ZEIG)");
  if (dim == 3 && !(flags & FPS_PLAN_CUBE_ZEIG) && n > 384)
    return fail(FPS_E_UNSUPPORTED, "the nested cube method is limited to n <= 384");
  fps_plan *pl = new (std::nothrow) fps_plan();
  if (!pl) return fail(FPS_E_NOMEM, "plan allocation failed");
  pl->dim = dim;
  pl->n = n;
  pl->tol = tol;
  pl->prec = prec;
  pl->out_basis = out_basis;
  pl->flags = flags;
  *out = pl;
  return FPS_OK;
}

std::vector<RefineRound> refine_schedule(double tol, bool dirichlet) {
  // Float rounds solve A~ dY + dY A~ = r_k to kRoundTol with every sweep
  // array stored in float.  On smooth right-hand sides such a round
  // contracts the error by about kContract (emulated at n = 64 .. 4096:
  // 5e-6 to 8e-6 per round, down to the FP64 level near 1e-14); the last
  // round only needs to take the error reached so far to tol, with a
  // factor 10 of margin.
  constexpr double kRoundTol = 1e-5, kContract = 1e-5;
  std::vector<RefineRound> t;
  double reached = 1.0;
  if (dirichlet && tol < kRoundTol) {
    // A Dirichlet lift puts O(1) content into every column of rows 0, 1 and
    // every row of columns 0, 1 of G; float rounds then contract by only
    // ~1e-3 after the first two (emulated: n = 1024, relative U error
    // 7.7e-6, 1.3e-9, 3.2e-12; the [0, 10] x [0, 1] box 5.9e-6, 9.6e-9, 1.9e-11).
    // Two float rounds leave <= ~5e-8 (symmetrized Y), and one FP64 round
    // finishes.
    t.push_back({kRoundTol, true});
    if (tol < 1e-9) t.push_back({kRoundTol, true});
    t.push_back({std::max(tol, std::min(kRoundTol, tol / 5e-8)), false});
    return t;
  }
  while (reached * kContract > tol * (1.0 + 1e-9)) {
    t.push_back({kRoundTol, true});
    reached *= kContract;
  }
  t.push_back({std::min(0.1, std::max(0.1 * tol / reached, tol)), true});
  return t;
}

// Square or rectangle plan (common fields, and for a rectangle rect / box /
// sx2 / sy2, already set): shifts, sweep tables, coefficient maps,
// workspace layout, and the device copies unless host-only.
fps_status plan2d_build(fps_plan *pl) {
  const int64_t n = pl->n;
  const int prec = pl->prec;
  const unsigned flags = pl->flags;
  const double tol = pl->tol;
  // Lemma B.1: sigma(A~) in [-1, -1/(30 n^4)]; sigma(B~) = sigma(-A~).
  const double delta = 1.0 / (30.0 * (double)n * (double)n * (double)n * (double)n);
  std::string err;
  double ea = -1.0, eb = -delta;  // enclosure of sigma(A~)
  if (flags & FPS_PLAN_TIGHT_SPECTRUM) spectrum_tight(n, &ea, &eb);
  // Theorem 2.1 intervals: sigma(A) in sx2 [ea, eb], sigma(B) in sy2 [-eb, -ea].
  // FP64: one ADI to tol.  FP32_REFINED: the rounds of refine_schedule(tol),
  // each an ADI to its own tolerance.
  const std::vector<RefineRound> sched =
      prec == FPS_FP32_REFINED ? refine_schedule(tol, (flags & FPS_PLAN_DIRICHLET) != 0)
                               : std::vector<RefineRound>{{tol, false}};
  pl->rtol.clear();
  pl->rf32.clear();
  for (const RefineRound &r : sched) {
    pl->rtol.push_back(r.tol);
    pl->rf32.push_back(r.f32 ? 1 : 0);
  }
  pl->rounds = (int)pl->rtol.size();
  pl->rsh.assign(pl->rtol.size(), fps::ShiftSet{});
  pl->rbase.assign(pl->rtol.size(), 0);
  int steps = 0;
  for (size_t k = 0; k < pl->rtol.size(); ++k) {
    fps::ShiftSet &sh = pl->rsh[k];
    if (!fps::zolotarev_shifts(pl->sx2 * ea, pl->sx2 * eb, -pl->sy2 * eb, -pl->sy2 * ea,
                               pl->rtol[k], sh, err))
      return fail(FPS_E_ARG, err);
    // Apply the steps in order of increasing |p_j| (the reverse of the
    // planner's order).  The J-step result does not depend on the order in
    // exact arithmetic (the error factors commute), but rounding does: a
    // small-shift step magnifies the rounding of its inputs by up to
    // ~ (sx2 + sy2) / |shift| in some modes, and the large-shift steps that
    // follow it damp those modes.  In the opposite order the symmetrized
    // iterate carries ~1e-10 relative error on Dirichlet-lift right-hand
    // sides (rows 0, 1 spanning every column mode) instead of ~1e-13, and
    // float storage (refinement rounds) stalls or diverges from n ~ 256 on.
    std::reverse(sh.p.begin(), sh.p.end());
    std::reverse(sh.q.begin(), sh.q.end());
    pl->rbase[k] = steps;
    steps += sh.J;
  }
  pl->shifts = pl->rsh[0];
  pl->n_f32 = 0;
  for (size_t k = 0; k < pl->rsh.size(); ++k)
    if (pl->rf32[k]) pl->n_f32 += pl->rsh[k].J;
  // Tables of every step of every round (a rectangle has two per step).
  std::vector<double> alpha, beta;
  for (const fps::ShiftSet &sh : pl->rsh)
    for (int j = 0; j < sh.J; ++j) {
      if (pl->rect) {  // tables 2j: sy2 A~ + p_j, 2j + 1: sx2 A~ - q_j
        alpha.push_back(pl->sy2);
        beta.push_back(sh.p[j]);
        alpha.push_back(pl->sx2);
        beta.push_back(-sh.q[j]);
      } else {
        alpha.push_back(1.0);
        beta.push_back(sh.p[j]);
      }
    }
  pl->L = fps::make_layout(n);
  fps::build_sweep_tables_ab(pl->L, alpha, beta, pl->tab, pl->ctab, nullptr, pl->l1);
  fps::build_conversions(pl->L, pl->Rs, pl->P);
  std::vector<double> RsA[2], RsB[2], PA[2], PB[2];
  for (int s = 0; s < 2; ++s) {
    const int64_t m = pl->L.m[s], mp = pl->L.mp[s], mo = pl->L.mo[s];
    const int64_t mop = (mo + fps::kPad - 1) / fps::kPad * fps::kPad;
    pl->mop[s] = mop;
    RsA[s].assign((size_t)mp * mp, 0.0);
    RsB[s].assign((size_t)mp * mp, 0.0);
    PA[s].assign((size_t)mop * mp, 0.0);
    PB[s].assign((size_t)mp * mop, 0.0);
    for (int64_t i = 0; i < m; ++i)
      for (int64_t k = 0; k < m; ++k) {
        RsA[s][(size_t)i * mp + k] = pl->Rs[s][(size_t)i * m + k];
        RsB[s][(size_t)k * mp + i] = pl->Rs[s][(size_t)i * m + k];
      }
    for (int64_t i = 0; i < mo; ++i)
      for (int64_t k = 0; k < m; ++k) {
        PA[s][(size_t)i * mp + k] = pl->P[s][(size_t)i * m + k];
        PB[s][(size_t)k * mop + i] = pl->P[s][(size_t)i * m + k];
      }
  }
  pl->sinv.resize(n);
  for (int64_t i = 0; i < n; ++i) pl->sinv[i] = 1.0 / std::sqrt((double)(i + 1) * (double)(i + 2));
  // A~ as a stencil along each parity block of the internal layout.
  pl->sdiag.assign(pl->L.npad, 0.0);
  pl->soff.assign(pl->L.npad, 0.0);
  for (int sp = 0; sp < 2; ++sp)
    for (int64_t k = 0; k < pl->L.m[sp]; ++k) {
      const int64_t r = sp * pl->L.mp[0] + k, i = 2 * k + sp;
      pl->sdiag[r] = fps::atilde_diag(i);
      if (k + 1 < pl->L.m[sp]) pl->soff[r] = fps::atilde_off(i);
    }

  const fps::Layout &L = pl->L;
  const int64_t sq = align256(L.npad * L.npad * 8);
  const int64_t lvb = align256(L.ncmax * 4 * L.npad * 8);  // [ncmax][2][2][npad]
  const int64_t abb = align256(2 * L.ncmax * L.npad * 2 * 8);  // [2][ncmax][npad][2]
  pl->off_G = 0;
  pl->off_GT = sq;
  pl->off_O0 = 2 * sq;
  pl->off_O1 = 3 * sq;
  pl->off_lv = 4 * sq;
  pl->off_ab = 4 * sq + lvb;
  const int64_t mobar = pl->mop[0] + pl->mop[1];
  pl->off_X = 4 * sq + lvb + abb;
  // second boundary-value buffer for sweeps that form their own carries
  // (chains of at most two chunks); after everything else
  const bool fused = L.ncmax <= 2;
  pl->ws_bytes = pl->off_X + align256(mobar * mobar * 8);
  if (prec == FPS_FP32_REFINED) {
    pl->off_R = pl->ws_bytes;  // r and r^T (batched solves), npad^2 floats each
    pl->ws_bytes += sq;
  }
  std::vector<double> lift[2];
  if (flags & FPS_PLAN_DIRICHLET) {
    fps::build_lift_map(L, lift);
    pl->off_bc = pl->ws_bytes;
    pl->ws_bytes += align256((4 * L.npad + 8) * 8);
  }
  pl->off_lv2 = pl->ws_bytes;
  pl->ws_bytes += lvb;
  pl->off_ab2 = pl->off_ab;
  if (!fused) {
    pl->off_ab2 = pl->ws_bytes;
    pl->ws_bytes += abb;
  }

  if (!(flags & FPS_PLAN_HOST_ONLY)) {
    fps_status s;
    if ((s = upload(pl->d_tab, pl->tab)) != FPS_OK || (s = upload(pl->d_ctab, pl->ctab)) != FPS_OK ||
        (s = upload(pl->d_l1, pl->l1)) != FPS_OK ||
        (s = upload(pl->d_RsA[0], RsA[0])) != FPS_OK || (s = upload(pl->d_RsA[1], RsA[1])) != FPS_OK ||
        (s = upload(pl->d_RsB[0], RsB[0])) != FPS_OK || (s = upload(pl->d_RsB[1], RsB[1])) != FPS_OK ||
        (s = upload(pl->d_PA[0], PA[0])) != FPS_OK || (s = upload(pl->d_PA[1], PA[1])) != FPS_OK ||
        (s = upload(pl->d_PB[0], PB[0])) != FPS_OK || (s = upload(pl->d_PB[1], PB[1])) != FPS_OK ||
        (s = upload(pl->d_sinv, pl->sinv)) != FPS_OK || (s = upload(pl->d_sdiag, pl->sdiag)) != FPS_OK ||
        (s = upload(pl->d_soff, pl->soff)) != FPS_OK ||
        (s = upload(pl->d_lift[0], lift[0])) != FPS_OK ||
        (s = upload(pl->d_lift[1], lift[1])) != FPS_OK)
      return s;
    // chains of more than two chunks: the two row-parity halves of the ADI
    // run on two streams (run_adi)
    if (!fused && L.m[1] > 0 && (s = create_side_stream(pl)) != FPS_OK) return s;
    pl->on_device = true;
  }
  return FPS_OK;
}

}  // namespace detail
}  // namespace fps

using namespace fps::detail;

extern "C" {

const char *fps_version(void) { return "fps 0.1 (gfx950)"; }

const char *fps_status_string(fps_status s) {
  switch (s) {
    case FPS_OK: return "ok";
    case FPS_E_ARG: return "invalid argument";
    case FPS_E_UNSUPPORTED: return "unsupported";
    case FPS_E_NOMEM: return "out of memory";
    case FPS_E_HIP: return "HIP runtime error";
    case FPS_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char *fps_last_error(void) { return last_error(); }

fps_status fps_adi_shifts(double a, double b, double c, double d, double tol, int cap, int *J,
                          double *p, double *q) {
  if (!J) return fail(FPS_E_ARG, "J must not be null");
  fps::ShiftSet S;
  std::string err;
  if (!fps::zolotarev_shifts(a, b, c, d, tol, S, err)) return fail(FPS_E_ARG, err);
  *J = S.J;
  if (cap < S.J) return fail(FPS_E_STATE, "cap smaller than J");
  if (!p || !q) return fail(FPS_E_ARG, "null output arrays");
  for (int j = 0; j < S.J; ++j) {
    p[j] = S.p[j];
    q[j] = S.q[j];
  }
  return FPS_OK;
}

fps_status fps_plan_create(fps_plan **out, int dim, int64_t n, int bc, double tol, int prec,
                           int out_basis, unsigned flags) {
  if (!out) return fail(FPS_E_ARG, "out must not be null");
  *out = nullptr;
  fps_plan *pl = nullptr;
  fps_status s = plan_common(&pl, dim, n, bc, tol, prec, out_basis, flags);
  if (s != FPS_OK) return s;
  if (dim == 3) {
    s = cube_plan_build(pl);
    if (s == FPS_OK && !(flags & FPS_PLAN_HOST_ONLY)) s = cube_plan_upload(pl);
    pl->on_device = s == FPS_OK && !(flags & FPS_PLAN_HOST_ONLY);
  } else {
    s = plan2d_build(pl);
  }
  if (s != FPS_OK) {
    delete pl;
    return s;
  }
  *out = pl;
  return FPS_OK;
}

fps_status fps_plan_create_cylinder(fps_plan **out, int64_t n, int64_t n_theta, unsigned flags) {
  if (!out) return fail(FPS_E_ARG, "out must not be null");
  *out = nullptr;
  if (flags & ~FPS_PLAN_HOST_ONLY) return fail(FPS_E_ARG, "cylinder plans take FPS_PLAN_HOST_ONLY only");
  fps_plan *pl = nullptr;
  fps_status s = plan_common(&pl, 3, n, FPS_BC_DIRICHLET_ZERO, 0.5, FPS_FP64, FPS_OUT_CHEB, flags);
  if (s != FPS_OK) return s;
  if ((s = cyl_plan_build(pl, n_theta)) == FPS_OK && !(flags & FPS_PLAN_HOST_ONLY))
    s = cyl_plan_upload(pl);
  if (s != FPS_OK) {
    delete pl;
    return s;
  }
  pl->on_device = !(flags & FPS_PLAN_HOST_ONLY);
  *out = pl;
  return FPS_OK;
}

fps_status fps_cylinder_mode_bands(int64_t n, int64_t k, double *P_host, double *Q_host) {
  if (n < 2 || (n & 1) || n > 512) return fail(FPS_E_ARG, "n must be even, 2 <= n <= 512");
  if (!P_host || !Q_host) return fail(FPS_E_ARG, "null output");
  std::vector<double> P, Q;
  cyl_mode_bands(n, k < 0 ? -k : k, P, Q);
  std::copy(P.begin(), P.end(), P_host);
  std::copy(Q.begin(), Q.end(), Q_host);
  return FPS_OK;
}

fps_status fps_plan_create_rect(fps_plan **out, int64_t n, const double *box, double tol, int prec,
                                int out_basis, unsigned flags) {
  if (!out) return fail(FPS_E_ARG, "out must not be null");
  *out = nullptr;
  if (!box) return fail(FPS_E_ARG, "box must not be null");
  const double a = box[0], b = box[1], c = box[2], d = box[3];
  if (!(std::isfinite(a) && std::isfinite(b) && std::isfinite(c) && std::isfinite(d)) ||
      !(b > a) || !(d > c))
    return fail(FPS_E_ARG, "box must be finite with a < b and c < d");
  const double sx = 2.0 / (b - a), sy = 2.0 / (d - c);
  if (!(std::isfinite(sx * sx) && std::isfinite(sy * sy) && sx * sx > 0.0 && sy * sy > 0.0))
    return fail(FPS_E_ARG, "box side lengths out of range");
  if (flags & FPS_PLAN_CUBE_ZEIG) return fail(FPS_E_ARG, "FPS_PLAN_CUBE_ZEIG applies to cube plans only");
  fps_plan *pl = nullptr;
  fps_status s = plan_common(&pl, 2, n, FPS_BC_DIRICHLET_ZERO, tol, prec, out_basis, flags);
  if (s != FPS_OK) return s;
  pl->rect = true;
  for (int i = 0; i < 4; ++i) pl->box[i] = box[i];
  pl->sx2 = sx * sx;
  pl->sy2 = sy * sy;
  if ((s = plan2d_build(pl)) != FPS_OK) {
    delete pl;
    return s;
  }
  *out = pl;
  return FPS_OK;
}

fps_status fps_plan_info(const fps_plan *pl, int *J, int64_t *ws_bytes, int64_t *out_entries) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (pl->cyl) {
    if (J) *J = 0;
    if (ws_bytes) *ws_bytes = cyl_ws_bytes(pl);
    if (out_entries) *out_entries = cyl_out_entries(pl);
    return FPS_OK;
  }
  if (J) *J = pl->shifts.J;
  if (ws_bytes) *ws_bytes = pl->ws_bytes;
  if (out_entries) {
    const int64_t e = pl->out_basis == FPS_OUT_NATIVE ? pl->n : pl->n + 2;
    *out_entries = pl->dim == 2 ? e * e : e * e * e;
  }
  return FPS_OK;
}

fps_status fps_plan_refinement(const fps_plan *pl, int *rounds, int *f32_steps) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (rounds) *rounds = pl->rounds;
  if (f32_steps) *f32_steps = pl->n_f32;
  return FPS_OK;
}

fps_status fps_plan_rounds(const fps_plan *pl, int *steps, double *tols, int cap) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  const bool zr = pl->zeig && pl->prec == FPS_FP32_REFINED;
  if (!zr && (pl->dim != 2 || pl->cyl))
    return fail(FPS_E_STATE, "rounds exist for square, rectangle and refined z-eigenbasis plans");
  for (int k = 0; k < pl->rounds && k < cap; ++k) {
    if (steps) steps[k] = zr ? pl->zrJmax[(size_t)k] : pl->rsh[(size_t)k].J;
    if (tols) tols[k] = pl->rtol[(size_t)k];
  }
  return FPS_OK;
}

fps_status fps_plan_inner_counts(const fps_plan *pl, int *counts, int cap) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (pl->dim != 3 || pl->zeig)
    return fail(FPS_E_STATE, "inner counts exist for nested-ADI cube plans only");
  if (!counts && cap > 0) return fail(FPS_E_ARG, "null output");
  for (int i = 0; i < pl->shifts.J && i < cap; ++i) counts[i] = pl->inner_J[i];
  return FPS_OK;
}

fps_status fps_plan_slice_counts(const fps_plan *pl, int *counts, int cap, int *count) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (!pl->zeig) return fail(FPS_E_STATE, "slice counts exist for z-eigenbasis cube plans only");
  const int K = (int)pl->zJ.size();
  if (count) *count = K;
  if (counts)
    for (int k = 0; k < K && k < cap; ++k) counts[k] = pl->zJ[k];
  return FPS_OK;
}

fps_status fps_plan_shifts(const fps_plan *pl, double *p) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (!p) return fail(FPS_E_ARG, "null output");
  for (int j = 0; j < pl->shifts.J; ++j) p[j] = pl->shifts.p[j];
  return FPS_OK;
}

fps_status fps_plan_shift_pairs(const fps_plan *pl, double *p, double *q) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (!p || !q) return fail(FPS_E_ARG, "null output");
  for (int j = 0; j < pl->shifts.J; ++j) {
    p[j] = pl->shifts.p[j];
    q[j] = pl->shifts.q[j];
  }
  return FPS_OK;
}

fps_status fps_solve_dirichlet(fps_plan *pl, const double *F, const double *bc, double *U, void *ws,
                               void *stream) {
  fps_status s = check_solve_args(pl, F, U, ws);
  if (s != FPS_OK) return s;
  if (!bc) return fail(FPS_E_ARG, "null pointer argument");
  if (pl->dim != 2) return fail(FPS_E_UNSUPPORTED, "Dirichlet data: square and rectangle plans only");
  if (pl->out_basis != FPS_OUT_CHEB)
    return fail(FPS_E_UNSUPPORTED, "Dirichlet data need the Chebyshev output basis");
  if (!(pl->flags & FPS_PLAN_DIRICHLET))
    return fail(FPS_E_STATE, "the plan was created without FPS_PLAN_DIRICHLET");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  if ((s = rhs_transform(pl, F, w, st, bc)) != FPS_OK) return s;
  double *Y = nullptr;
  if ((s = solve_symmetric(pl, w, st, &Y)) != FPS_OK) return s;
  if ((s = out_transform(pl, Y, U, w, st)) != FPS_OK) return s;
  FPS_HIP(fps::launch_bc_lift_out(U, bc, (const double *)(w + pl->off_bc), pl->L.n, pl->L.npad, st));
  return FPS_OK;
}

fps_status fps_solve(fps_plan *pl, const double *F, double *U, void *ws, void *stream) {
  fps_status s = check_solve_args(pl, F, U, ws);
  if (s != FPS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  const fps::Layout &L = pl->L;
  if (pl->cyl) return cyl_solve(pl, F, U, w, st);
  if (pl->dim == 3) return cube_solve(pl, F, U, w, st);
  if ((s = rhs_transform(pl, F, w, st)) != FPS_OK) return s;
  double *Y = nullptr;
  if ((s = solve_symmetric(pl, w, st, &Y)) != FPS_OK) return s;
  if (pl->out_basis == FPS_OUT_NATIVE) {
    FPS_HIP(fps::launch_permute_out(Y, U, L.n, L.npad, L.mp[0], (const double *)pl->d_sinv.p, st));
    return FPS_OK;
  }
  return out_transform(pl, Y, U, w, st);
}

fps_status fps_adi_native(fps_plan *pl, const double *G, double *Y, void *ws, void *stream) {
  fps_status s = check_solve_args(pl, G, Y, ws);
  if (s != FPS_OK) return s;
  if (pl->dim != 2 || pl->prec != FPS_FP64)
    return fail(FPS_E_UNSUPPORTED, "the J-step iterate entry point needs a square FP64 plan");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  const fps::Layout &L = pl->L;
  double *Gp = (double *)(w + pl->off_G);
  FPS_HIP(fps::launch_permute_in(G, Gp, L.n, L.npad, L.mp[0], st));
  if ((s = run_adi(pl, pl->shifts, 0, Gp, 0, 0, w + pl->off_O0, w + pl->off_O1, w, st)) != FPS_OK)
    return s;
  const int J = pl->shifts.J;
  FPS_HIP(fps::launch_finalize<double>((double *)(w + pl->off_O1), (double *)(w + pl->off_ab),
                                       pl->tab_dev(pl->tab2(J - 1)), Y, 1, nullptr, L.n, L.npad, L.mp[0],
                                       L.mstride, L.ncmax, st));
  return FPS_OK;
}

}  // extern "C"

namespace fps {
namespace detail {

// The adjoint's steps around the ADI map (Frobenius transposes of the input
// and output maps, Sec. 3.4 and Table 1 read backwards).
//
// GEMMs of the adjoint's input map (Chebyshev output basis): Ybar_st =
// P_s^T Ubar_st P_t per parity block, from Ubar in the parity-blocked
// layout (X region, mobar x mobar) through temporaries in O0/O1, into G.
int adj_in_gemms(const fps_plan *pl, char *w, fps::GemmProb *g1, fps::GemmProb *g2) {
  const fps::Layout &L = pl->L;
  const int64_t npad = L.npad;
  const int64_t mo0 = pl->mop[0], mobar = pl->mop[0] + pl->mop[1];
  const double *Up = (const double *)(w + pl->off_X);
  double *G = (double *)(w + pl->off_G);
  double *Tt = (double *)(w + pl->off_O0);  // temporaries mop_s x mp_t
  int cnt = 0;
  int64_t toff = 0;
  for (int s2 = 0; s2 < 2; ++s2)
    for (int t = 0; t < 2; ++t) {
      const int64_t ms = L.mp[s2], mt = L.mp[t], mos = pl->mop[s2], mot = pl->mop[t];
      if (L.m[s2] == 0 || L.m[t] == 0) continue;
      double *Tst = Tt + toff;
      toff += mos * mt;
      // T_st = Ubar_st P_t; B(k, j) = P_t[k][j] = 0 for k > j + 1.
      g1[cnt] = fps::GemmProb{Up + (s2 * mo0) * mobar + t * mo0, (const double *)pl->d_PA[t].p,
                              Tst, mos, mt, mot, mobar, 1, mt, 1, mt, 1, 0, 0, 0, 0, 0, 0, 1, 1};
      // Ybar_st = P_s^T T_st; A(i, k) = P_s[k][i] = 0 for k > i + 1.
      g2[cnt] = fps::GemmProb{(const double *)pl->d_PB[s2].p, Tst,
                              G + (s2 * L.mp[0]) * npad + t * L.mp[0], ms, mt, mos, mos, 1, mt, 1,
                              npad, 1, 0, 0, 0, 0, 1, 1, 0, 0};
      ++cnt;
    }
  return cnt;
}

// GEMMs of the adjoint's output map: Fbar = R^T S^-1 Gbar S^-1 R, blockwise
// Rs_s^T Gbar_st Rs_t into the strided view of Fbar (Gbar: the ADI output,
// parity-blocked), through temporaries in O0/O1.
int adj_out_gemms(const fps_plan *pl, const double *Yb, double *Fbar, char *w, fps::GemmProb *g1,
                  fps::GemmProb *g2) {
  const fps::Layout &L = pl->L;
  const int64_t n = L.n, npad = L.npad;
  double *Tb = (double *)(w + pl->off_O0);
  int cnt = 0;
  int64_t toff = 0;
  for (int s2 = 0; s2 < 2; ++s2)
    for (int t = 0; t < 2; ++t) {
      const int64_t ms = L.mp[s2], mt = L.mp[t];
      if (L.m[s2] == 0 || L.m[t] == 0) continue;
      double *Tst = Tb + toff;
      toff += ms * mt;
      // T_st = Gbar_st Rs_t; B(k, j) = Rs_t[k][j] = 0 for k > j.
      g1[cnt] = fps::GemmProb{Yb + (s2 * L.mp[0]) * npad + t * L.mp[0], (const double *)pl->d_RsA[t].p,
                              Tst, ms, mt, mt, npad, 1, mt, 1, mt, 1, 0, 0, 0, 0, 0, 0, 1, 0};
      // Fbar_st = Rs_s^T T_st; A(i, k) = Rs_s[k][i] = 0 for k > i.
      g2[cnt] = fps::GemmProb{(const double *)pl->d_RsB[s2].p, Tst, Fbar + s2 * n + t, L.m[s2],
                              L.m[t], ms, ms, 1, mt, 1, 2 * n, 2, 0, 0, 0, 0, 1, 0, 0, 0};
      ++cnt;
    }
  return cnt;
}

// The adjoint's input map up to its GEMMs: Ubar permuted into the
// parity-blocked layout and G cleared (Chebyshev output), or Ybar = S^-1
// Xbar S^-1 straight into G (native output).
fps_status adjoint_in_pre(const fps_plan *pl, const double *Ubar, char *w, hipStream_t st) {
  const fps::Layout &L = pl->L;
  const int64_t n = L.n, npad = L.npad, N = n + 2;
  double *G = (double *)(w + pl->off_G);
  if (pl->out_basis == FPS_OUT_NATIVE) {
    FPS_HIP(fps::launch_permute_in(Ubar, G, n, npad, L.mp[0], st, (const double *)pl->d_sinv.p));
    return FPS_OK;
  }
  const int64_t mo0 = pl->mop[0], mobar = pl->mop[0] + pl->mop[1];
  if (npad * mobar * 8 > pl->off_lv - pl->off_O0)
    return fail(FPS_E_STATE, "internal: adjoint temporaries exceed workspace");
  FPS_HIP(fps::launch_permute_in(Ubar, (double *)(w + pl->off_X), N, mobar, mo0, st));
  FPS_HIP(fps::launch_fill(G, npad * npad, 0.0, st));
  return FPS_OK;
}

// adjoint_in: Ybar into G from Ubar.
fps_status adjoint_in(const fps_plan *pl, const double *Ubar, char *w, hipStream_t st) {
  fps_status s;
  if ((s = adjoint_in_pre(pl, Ubar, w, st)) != FPS_OK) return s;
  if (pl->out_basis != FPS_OUT_NATIVE) {
    fps::GemmProb g1[4], g2[4];
    const int cnt = adj_in_gemms(pl, w, g1, g2);
    FPS_HIP(fps::launch_gemm(g1, cnt, st));
    FPS_HIP(fps::launch_gemm(g2, cnt, st));
  }
  return FPS_OK;
}

// adjoint_out: Fbar from the ADI output Gbar.
fps_status adjoint_out(const fps_plan *pl, const double *Yb, double *Fbar, char *w,
                       hipStream_t st) {
  fps::GemmProb g1[4], g2[4];
  const int cnt = adj_out_gemms(pl, Yb, Fbar, w, g1, g2);
  FPS_HIP(fps::launch_gemm(g1, cnt, st));
  FPS_HIP(fps::launch_gemm(g2, cnt, st));
  return FPS_OK;
}

}  // namespace detail
}  // namespace fps

extern "C" {

fps_status fps_solve_adjoint(fps_plan *pl, const double *Ubar, double *Fbar, void *ws,
                             void *stream) {
  fps_status s = check_solve_args(pl, Ubar, Fbar, ws);
  if (s != FPS_OK) return s;
  if (pl->dim != 2 || pl->prec != FPS_FP64)
    return fail(FPS_E_UNSUPPORTED, "adjoint: square FP64 plans only");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  if ((s = fps::detail::adjoint_in(pl, Ubar, w, st)) != FPS_OK) return s;
  double *Yb = nullptr;
  if ((s = solve_symmetric(pl, w, st, &Yb)) != FPS_OK) return s;  // Gbar, in G
  return fps::detail::adjoint_out(pl, Yb, Fbar, w, st);
}

fps_status fps_plan_set_sweep_timing(fps_plan *pl, int capacity) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (capacity < 0) return fail(FPS_E_ARG, "capacity must be >= 0");
  if (!pl->on_device) return fail(FPS_E_STATE, "plan was created host-only");
  release_events(pl);
  for (int i = 0; i < 2 * capacity; ++i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      release_events(pl);
      return fail(FPS_E_HIP, "hipEventCreate failed");
    }
    pl->ev.push_back(e);
  }
  return FPS_OK;
}

fps_status fps_plan_sweep_time(fps_plan *pl, double *ms_host, int64_t cap, int64_t *launches) {
  if (!valid_plan(pl)) return fail(FPS_E_STATE, "invalid or destroyed plan");
  if (!launches || (cap > 0 && !ms_host)) return fail(FPS_E_ARG, "null output");
  for (int64_t i = 0; i < pl->ev_used; ++i) {
    FPS_HIP(hipEventSynchronize(pl->ev[2 * i + 1]));
    float ms = 0.0f;
    FPS_HIP(hipEventElapsedTime(&ms, pl->ev[2 * i], pl->ev[2 * i + 1]));
    if (i < cap) ms_host[i] = ms;
  }
  *launches = pl->ev_used;
  pl->ev_used = 0;
  return FPS_OK;
}

void fps_plan_destroy(fps_plan *pl) {
  if (!valid_plan(pl)) return;
  release_events(pl);
  if (pl->zside) (void)hipStreamDestroy(pl->zside);
  if (pl->zfork) (void)hipEventDestroy(pl->zfork);
  if (pl->zjoin) (void)hipEventDestroy(pl->zjoin);
  pl->magic = 0;
  delete pl;
}

}  // extern "C"
