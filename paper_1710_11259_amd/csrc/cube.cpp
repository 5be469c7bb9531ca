// Poisson on the cube [-1,1]^3 (Sec. 5): the two-level nested ADI.
//
// In symmetric variables the cube system (5.2) reads
//   (A~ x A~ x I + A~ x I x A~ + I x A~ x A~) Y = -G,  G = (S^-1)^{x3} F_C,
// and with K = -A~^-1 (symmetric positive definite, spectrum in
// [1, 1/delta], Lemma B.1) it becomes (K_x + K_y + K_z) Y = B with
// B = (A~^-1)^{x3} G.  The outer ADI (Algorithm 2 for (-H) Y - Y V = -B,
// H = K_x + K_y, V = K_z) alternates a z half-step, one z-fiber sweep, with
// an (x, y) half-step (H + q) Y = R that is, on every z-slice, the symmetric
// Sylvester equation (K + q/2) Y + Y (K + q/2) = R, solved by an inner
// Algorithm 2 to a tighter tolerance (the paper's nesting (5.3)-(5.9) with
// its innermost level replaced by banded solves).  Every shifted operator
// (K + s I)^-1 = (I - s A~)^-1 (-A~) is "multiply by the tridiagonal A~,
// then solve with the tridiagonal I - s A~" along one direction, which is
// what the stencil form of the sweep kernel does.
//
// Pass form.  Outer step i with shifts (p_i, q_i), zR_i = -B + (H + p_i) Y_i:
//   z sweep:   x = (I + p_i A~)^-1 A~ zR_i along z  (Y_{i+1/2} = -x),
//              R_i = zR_i + B + (q_i - p_i) x = B + (V - q_i) Y_{i+1/2};
//   inner:     the square pass form with A~ replaced by -(K + q_i/2) and G by
//              -R_i, solving (K + q_i/2 - p) = -(I - (q_i/2 - p) A~)^-1 A~...;
//   finalize:  zR_{i+1} = -B + R_i + (p_{i+1} - q_i) Y_{i+1}.
// With parity blocks of at most 128 the inner ADI of an outer step runs as
// one launch of the slice kernel of zeig_lds.hip, every slice block held in
// LDS for all its inner steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "solver.hpp"

namespace fps {
namespace detail {

namespace {

// Sizes [z][y][x] of one stage of the coefficient maps and the offset of
// the parity-1 block on every axis.
struct Dims {
  int64_t d[3];
  int64_t b0[3];
};

// GEMM problems of out = M along axis `mode` (0: z, 1: y, 2: x) of `in`,
// one per parity s (and per z-slice for mode 1).  MA[s] is M_s row-major
// (N[s] rows, row stride lda[s]); MB[s] is M_s^T row-major (K[s] rows, row
// stride ldb[s]).
void mode_probs(const double *in, const Dims &di, double *out, const Dims &dout, int mode,
                const double *const MA[2], const int64_t lda[2], const double *const MB[2],
                const int64_t ldb[2], const int64_t N[2], const int64_t K[2],
                std::vector<fps::GemmProb> &probs) {
  for (int s = 0; s < 2; ++s) {
    if (N[s] == 0 || K[s] == 0) continue;
    if (mode == 2) {
      probs.push_back(fps::GemmProb{in + s * di.b0[2], MB[s], out + s * dout.b0[2],
                                    di.d[0] * di.d[1], N[s], K[s], di.d[2], 1, ldb[s], 1,
                                    dout.d[2], 1, 0, 0, 0, 0, 0, 0, 0, 0});
    } else if (mode == 0) {
      const int64_t pin = di.d[1] * di.d[2], pout = dout.d[1] * dout.d[2];
      probs.push_back(fps::GemmProb{MA[s], in + s * di.b0[0] * pin, out + s * dout.b0[0] * pout,
                                    N[s], pin, K[s], lda[s], 1, pin, 1, pout, 1, 0, 0, 0, 0, 0,
                                    0, 0, 0});
    } else {
      for (int64_t z = 0; z < di.d[0]; ++z)
        probs.push_back(fps::GemmProb{
            MA[s], in + z * di.d[1] * di.d[2] + s * di.b0[1] * di.d[2],
            out + z * dout.d[1] * dout.d[2] + s * dout.b0[1] * dout.d[2], N[s], di.d[2], K[s],
            lda[s], 1, di.d[2], 1, dout.d[2], 1, 0, 0, 0, 0, 0, 0, 0, 0});
    }
  }
}

fps_status launch_probs(const std::vector<fps::GemmProb> &probs, hipStream_t st) {
  for (size_t i = 0; i < probs.size(); i += 4)
    FPS_HIP(fps::launch_gemm(probs.data() + i, (int)std::min<size_t>(4, probs.size() - i), st));
  return FPS_OK;
}

// Device GEMM table of mode-y problems whose `in` / `out` are workspace
// offsets (A absolute, B and C workspace-relative).
fps_status upload_table(const std::vector<fps::GemmProb> &probs, DeviceBuf &d, DeviceBuf &map,
                        int &tiles) {
  std::vector<fps::GemmDesc> tab;
  tiles = 0;
  for (const fps::GemmProb &q : probs) {
    if (!fps::gemm_operands_ok(q)) return fail(FPS_E_STATE, "internal: cube GEMM operand layout");
    fps::GemmDesc e{q, 0, 1, 1, tiles, 0};
    tiles += fps::gemm_tiles(q, &e.ntx);
    tab.push_back(e);
  }
  fps_status s;
  if ((s = upload(d, tab)) != FPS_OK || (s = upload(map, fps::gemm_table_map(tab))) != FPS_OK)
    return s;
  return FPS_OK;
}

Dims full_dims(const fps::Layout &L) {
  return Dims{{L.npad, L.npad, L.npad}, {L.mp[0], L.mp[0], L.mp[0]}};
}

}  // namespace

fps_status zeig_build(fps_plan *pl);
fps_status zeig_upload(fps_plan *pl);
fps_status zeig_solve(fps_plan *pl, const double *F, double *U, char *w, hipStream_t st);

fps_status cube_plan_build(fps_plan *pl) {
  if (pl->flags & FPS_PLAN_CUBE_ZEIG) return zeig_build(pl);
  const int64_t n = pl->n;
  const double delta = 1.0 / (30.0 * (double)n * (double)n * (double)n * (double)n);
  // sigma(K) = -1 / sigma(A~) in [klo, khi]: [1, 1/delta] from Lemma B.1, or
  // from the computed extreme eigenvalues.
  double klo = 1.0, khi = 1.0 / delta;
  if (pl->flags & FPS_PLAN_TIGHT_SPECTRUM) {
    double a, b;
    spectrum_tight(n, &a, &b);
    klo = -1.0 / a;
    khi = -1.0 / b;
  }
  std::string err;
  if (!fps::zolotarev_shifts(-2.0 * khi, -2.0 * klo, klo, khi, pl->tol, pl->shifts, err))
    return fail(FPS_E_ARG, err);
  // The outer iteration needs its (x, y) half-steps solved well below its
  // own tolerance.
  pl->cube_inner_tol = pl->tol * 0.1;
  const int J1 = pl->shifts.J;
  std::vector<double> alpha, beta;
  for (int i = 0; i < J1; ++i) {  // z sweeps: I + p_i A~ (p_i < 0)
    alpha.push_back(pl->shifts.p[i]);
    beta.push_back(1.0);
  }
  pl->inner_J.assign(J1, 0);
  pl->inner_off.assign(J1, 0);
  pl->inner_p.clear();
  for (int i = 0; i < J1; ++i) {
    const double c = 0.5 * pl->shifts.q[i];
    fps::ShiftSet in;
    if (!fps::zolotarev_shifts(-(khi + c), -(klo + c), klo + c, khi + c, pl->cube_inner_tol, in,
                               err))
      return fail(FPS_E_ARG, err);
    pl->inner_J[i] = in.J;
    pl->inner_off[i] = (int)pl->inner_p.size();
    for (int j = 0; j < in.J; ++j) {  // inner sweeps: I - (c - p) A~
      pl->inner_p.push_back(in.p[j]);
      alpha.push_back(in.p[j] - c);
      beta.push_back(1.0);
    }
  }
  pl->L = fps::make_layout(n);
  const fps::Layout &L = pl->L;
  fps::build_sweep_tables_ab(L, alpha, beta, pl->tab, pl->ctab, nullptr, pl->l1);
  fps::build_conversions(L, pl->Rs, pl->P);
  for (int s = 0; s < 2; ++s) {
    pl->mop[s] = (L.mo[s] + fps::kPad - 1) / fps::kPad * fps::kPad;
    pl->mqc[s] = (L.mo[s] + 1) / 2 * 2;
  }
  pl->sinv.resize(n);
  for (int64_t i = 0; i < n; ++i) pl->sinv[i] = 1.0 / std::sqrt((double)(i + 1) * (double)(i + 2));
  pl->sdiag.assign(L.npad, 0.0);
  pl->soff.assign(L.npad, 0.0);
  for (int sp = 0; sp < 2; ++sp)
    for (int64_t k = 0; k < L.m[sp]; ++k) {
      const int64_t r = sp * L.mp[0] + k, i = 2 * k + sp;
      pl->sdiag[r] = fps::atilde_diag(i);
      if (k + 1 < L.m[sp]) pl->soff[r] = fps::atilde_off(i);
    }
  // Workspace: B, ZR, RX, RX^T, O0, O1 (npad^3 each), then lv and ab sized
  // for the npad^2 chains of a z sweep (also the npad slices x npad chains
  // of the inner sweeps).
  const int64_t vol = align256(L.npad * L.npad * L.npad * 8);
  const int64_t ch = L.npad * L.npad;
  pl->off_G = 0;
  pl->off_ZR = vol;
  pl->off_RX = 2 * vol;
  pl->off_RXT = 3 * vol;
  pl->off_O0 = 4 * vol;
  pl->off_O1 = 5 * vol;
  pl->off_lv = 6 * vol;
  pl->off_ab = pl->off_lv + align256(L.ncmax * 4 * ch * 8);
  pl->ws_bytes = pl->off_ab + align256(2 * L.ncmax * ch * 2 * 8);
  // output temporaries: [npad][npad][mq] and [mq]^3 in O0..O1, [npad][mq][mq] in RX..RX^T
  const int64_t mq = pl->mqc[0] + pl->mqc[1];
  if (L.npad * L.npad * mq * 8 > 2 * vol || mq * mq * mq * 8 > 2 * vol ||
      L.npad * mq * mq * 8 > 2 * vol)
    return fail(FPS_E_STATE, "internal: cube output temporaries exceed the workspace");
  return FPS_OK;
}

fps_status cube_plan_upload(fps_plan *pl) {
  if (pl->zeig) return zeig_upload(pl);
  const fps::Layout &L = pl->L;
  fps_status s;
  // Input map blocks Rb_s = A~_s^-1 (S^-1 R)_s, zero padded to mp x mp, and
  // their transposes; output map blocks P_s (mop x mp) and P_s^T (mp x mop).
  std::vector<double> RbA[2], RbB[2], PA[2], PB[2];
  for (int sp = 0; sp < 2; ++sp) {
    const int64_t m = L.m[sp], mp = L.mp[sp], mo = L.mo[sp], mop = pl->mop[sp];
    RbA[sp].assign((size_t)mp * mp, 0.0);
    RbB[sp].assign((size_t)mp * mp, 0.0);
    PA[sp].assign((size_t)mop * mp, 0.0);
    PB[sp].assign((size_t)mp * mop, 0.0);
    // Thomas factors of A~ restricted to parity sp (negative definite).
    std::vector<long double> ib(m), l(m), col(m);
    for (int64_t k = 0; k < m; ++k) {
      const long double d = fps::atilde_diag(2 * k + sp);
      if (k == 0) {
        ib[k] = 1.0L / d;
      } else {
        const long double e = fps::atilde_off(2 * (k - 1) + sp);
        l[k] = e * ib[k - 1];
        ib[k] = 1.0L / (d - l[k] * e);
      }
    }
    for (int64_t b = 0; b < m; ++b) {
      for (int64_t k = 0; k < m; ++k) col[k] = pl->Rs[sp][(size_t)k * m + b];
      for (int64_t k = 1; k < m; ++k) col[k] -= l[k] * col[k - 1];
      col[m - 1] *= ib[m - 1];
      for (int64_t k = m - 2; k >= 0; --k)
        col[k] = (col[k] - (long double)fps::atilde_off(2 * k + sp) * col[k + 1]) * ib[k];
      for (int64_t a = 0; a < m; ++a) {
        RbA[sp][(size_t)a * mp + b] = (double)col[a];
        RbB[sp][(size_t)b * mp + a] = (double)col[a];
      }
    }
    for (int64_t i = 0; i < mo; ++i)
      for (int64_t k = 0; k < m; ++k) {
        PA[sp][(size_t)i * mp + k] = pl->P[sp][(size_t)i * m + k];
        PB[sp][(size_t)k * mop + i] = pl->P[sp][(size_t)i * m + k];
      }
  }
  std::vector<double> pre(pl->sdiag);
  pre.insert(pre.end(), pl->soff.begin(), pl->soff.end());
  if ((s = upload(pl->d_tab, pl->tab)) != FPS_OK || (s = upload(pl->d_ctab, pl->ctab)) != FPS_OK ||
      (s = upload(pl->d_l1, pl->l1)) != FPS_OK ||
      (s = upload(pl->d_RbA[0], RbA[0])) != FPS_OK || (s = upload(pl->d_RbA[1], RbA[1])) != FPS_OK ||
      (s = upload(pl->d_RbB[0], RbB[0])) != FPS_OK || (s = upload(pl->d_RbB[1], RbB[1])) != FPS_OK ||
      (s = upload(pl->d_PA[0], PA[0])) != FPS_OK || (s = upload(pl->d_PA[1], PA[1])) != FPS_OK ||
      (s = upload(pl->d_PB[0], PB[0])) != FPS_OK || (s = upload(pl->d_PB[1], PB[1])) != FPS_OK ||
      (s = upload(pl->d_sinv, pl->sinv)) != FPS_OK || (s = upload(pl->d_pre, pre)) != FPS_OK)
    return s;
  // Mode-y GEMM tables over workspace offsets.
  const Dims full = full_dims(L);
  const int64_t K[2] = {L.mp[0], L.mp[1]};
  {
    const double *MA[2] = {(const double *)pl->d_RbA[0].p, (const double *)pl->d_RbA[1].p};
    const int64_t lda[2] = {L.mp[0], L.mp[1]};
    const int64_t N[2] = {L.m[0] > 0 ? L.mp[0] : 0, L.m[1] > 0 ? L.mp[1] : 0};
    std::vector<fps::GemmProb> probs;
    mode_probs((const double *)(intptr_t)pl->off_O1, full, (double *)(intptr_t)pl->off_O0, full, 1,
               MA, lda, nullptr, lda, N, K, probs);
    if ((s = upload_table(probs, pl->d_gy_in, pl->d_gy_map_in, pl->gy_tiles[0])) != FPS_OK)
      return s;
  }
  {
    const int64_t mq = pl->mqc[0] + pl->mqc[1];
    const Dims di{{L.npad, L.npad, mq}, {L.mp[0], L.mp[0], pl->mqc[0]}};
    const Dims dout{{L.npad, mq, mq}, {L.mp[0], pl->mqc[0], pl->mqc[0]}};
    const double *MA[2] = {(const double *)pl->d_PA[0].p, (const double *)pl->d_PA[1].p};
    const int64_t lda[2] = {L.mp[0], L.mp[1]};
    const int64_t N[2] = {L.m[0] > 0 ? L.mo[0] : 0, L.m[1] > 0 ? L.mo[1] : 0};
    std::vector<fps::GemmProb> probs;
    mode_probs((const double *)(intptr_t)pl->off_O0, di, (double *)(intptr_t)pl->off_RX, dout, 1,
               MA, lda, nullptr, lda, N, K, probs);
    if ((s = upload_table(probs, pl->d_gy_out, pl->d_gy_map_out, pl->gy_tiles[1])) != FPS_OK)
      return s;
  }
  // The LDS-resident inner ADI: chunk multipliers of every table and, per
  // outer step, the sigmas of its inner steps (v - 2 p_j x along x, then
  // v - (p_j + p_{j+1}) x along y; the last y solve keeps x).
  pl->nlds = pl->prec == FPS_FP64 && fps::zeig_lds_fits(L.m[0], L.m[1]) && L.mp[0] <= 128 &&
             L.npad - L.mp[0] <= 128 && L.mstride % fps::kZeigLdsChunk == 0;
  if (pl->nlds) {
    std::vector<double> t32, c32, sg;
    fps::build_chunk_tables(L, pl->tab, fps::kZeigLdsChunk, t32, c32);
    for (int i = 0; i < pl->shifts.J; ++i) {
      const double *p2 = pl->inner_p.data() + pl->inner_off[i];
      const int J2 = pl->inner_J[i];
      for (int j = 0; j < J2; ++j) {
        sg.push_back(2.0 * p2[j]);
        sg.push_back(j + 1 < J2 ? p2[j] + p2[j + 1] : 0.0);
      }
    }
    if (sg.empty()) sg.push_back(0.0);
    if ((s = upload(pl->d_zl_tab32, t32)) != FPS_OK ||
        (s = upload(pl->d_zl_ctab32, c32)) != FPS_OK || (s = upload(pl->d_zl_sig, sg)) != FPS_OK)
      return s;
  }
  return FPS_OK;
}

fps_status cube_solve(fps_plan *pl, const double *F, double *U, char *w, hipStream_t st) {
  if (pl->zeig) return zeig_solve(pl, F, U, w, st);
  const fps::Layout &L = pl->L;
  const int64_t npad = L.npad, ch = npad * npad, mp0 = L.mp[0];
  double *B = (double *)(w + pl->off_G), *ZR = (double *)(w + pl->off_ZR);
  double *RX = (double *)(w + pl->off_RX), *RXT = (double *)(w + pl->off_RXT);
  double *O0 = (double *)(w + pl->off_O0), *O1 = (double *)(w + pl->off_O1);
  double *lv = (double *)(w + pl->off_lv), *ab = (double *)(w + pl->off_ab);
  const Dims full = full_dims(L);
  const int64_t K[2] = {L.mp[0], L.mp[1]};
  const int64_t ldm[2] = {L.mp[0], L.mp[1]};
  fps_status s;

  // Input map: B = F_T x_i (A~^-1 S^-1 R) on every axis.
  FPS_HIP(fps::launch_permute3_in(F, O0, L.n, npad, mp0, st));
  {
    const double *MA[2] = {(const double *)pl->d_RbA[0].p, (const double *)pl->d_RbA[1].p};
    const double *MB[2] = {(const double *)pl->d_RbB[0].p, (const double *)pl->d_RbB[1].p};
    const int64_t N[2] = {L.m[0] > 0 ? L.mp[0] : 0, L.m[1] > 0 ? L.mp[1] : 0};
    std::vector<fps::GemmProb> px, pz;
    mode_probs(O0, full, O1, full, 2, MA, ldm, MB, ldm, N, K, px);
    if ((s = launch_probs(px, st)) != FPS_OK) return s;
    FPS_HIP(fps::launch_gemm_table((const fps::GemmDesc *)pl->d_gy_in.p,
                                   (const int *)pl->d_gy_map_in.p, pl->gy_tiles[0], w, nullptr, st));
    mode_probs(O0, full, B, full, 0, MA, ldm, MB, ldm, N, K, pz);
    if ((s = launch_probs(pz, st)) != FPS_OK) return s;
  }

  const int J1 = pl->shifts.J;
  const std::vector<double> &p1 = pl->shifts.p, &q1 = pl->shifts.q;
  const double *pre = (const double *)pl->d_pre.p;
  fps::SweepArgs Z{};
  Z.npad = npad;
  Z.mp0 = L.mp[0];
  Z.mp1 = L.mp[1];
  Z.mstride = L.mstride;
  Z.ncmax = L.ncmax;
  Z.nc0 = (int)L.nc[0];
  Z.nc1 = (int)L.nc[1];
  Z.lv = lv;
  Z.pre = pre;
  fps::SweepArgs S = Z;  // per-slice sweeps
  Z.ncols = ch;
  Z.ld = ch;
  Z.nbatch = 1;
  S.ncols = npad;
  S.ld = npad;
  S.nbatch = (int)npad;
  S.bstride = ch;
  S.lvb = L.ncmax * 4 * npad;
  S.abb = 2 * L.ncmax * npad * 2;
  for (int i = 0; i < J1; ++i) {
    // z half-step
    Z.in = i == 0 ? (const void *)B : (const void *)ZR;
    Z.in_scale = i == 0 ? -1.0 : 1.0;
    Z.g = B;
    Z.sg = 0.0;
    Z.og = 1.0;
    Z.tab = pl->tab_dev(i);
    Z.l1 = pl->l1_dev(i);
    Z.sigma = p1[i] - q1[i];
    Z.out = O0;
    Z.out_mode = 2;
    FPS_HIP(timed_sweep(pl, Z, st));
    FPS_HIP(fps::launch_reduce(lv, pl->ctab_dev(i), ab, -Z.sigma, ch, Z.nc0, Z.nc1, L.ncmax, st));
    // (the LDS-resident inner ADI reads R in place: no per-slice transpose)
    FPS_HIP(fps::launch_cube_zfinal(O0, ab, pl->tab_dev(i), RX, pl->nlds ? nullptr : RXT, npad, mp0,
                                    L.mstride, L.ncmax, st));
    // (x, y) half-step: inner ADI on every z-slice
    const int J2 = pl->inner_J[i];
    const double *p2 = pl->inner_p.data() + pl->inner_off[i];
    const int t0 = J1 + pl->inner_off[i];
    if (pl->nlds) {
      // every slice's inner ADI in one launch, each parity block resident
      // in one workgroup's LDS; its epilogue forms the next outer step's
      // zR (the update of k_cube_ifinal) from the complete final x
      fps::ZeigLdsArgs za{};
      za.G = RX;
      za.Y = ZR;
      za.B = i + 1 < J1 ? B : nullptr;
      za.cy = i + 1 < J1 ? p1[i + 1] - q1[i] : 1.0;
      za.cr = 1.0;
      za.cb = -1.0;
      za.tab = (const double *)pl->d_tab.p;
      za.tab32 = (const double *)pl->d_zl_tab32.p;
      za.ctab32 = (const double *)pl->d_zl_ctab32.p;
      za.pre = pre;
      za.sig = (const double *)pl->d_zl_sig.p + 2 * (int64_t)pl->inner_off[i];
      za.npad = npad;
      za.mp0 = mp0;
      za.mstride = L.mstride;
      za.ncmax = L.ncmax;
      za.m0 = (int)L.m[0];
      za.m1 = (int)L.m[1];
      za.tab0_all = t0;
      za.J_all = J2;
      const bool tm = pl->ev_used * 2 + 1 < (int64_t)pl->ev.size();
      FPS_HIP(fps::launch_zeig_lds(za, (int)npad, st, tm ? pl->ev[2 * pl->ev_used] : nullptr,
                                   tm ? pl->ev[2 * pl->ev_used + 1] : nullptr, true));
      if (tm) ++pl->ev_used;
    } else {
      for (int j = 0; j < J2; ++j) {
        const int t = t0 + j;
        const bool last = j == J2 - 1;
        fps::SweepArgs a = S;
        a.in = j == 0 ? (const void *)RXT : (const void *)O1;
        a.in_scale = 1.0;
        a.ab_prev = j == 0 ? nullptr : ab;
        a.tab_prev = j == 0 ? nullptr : pl->tab_dev(t - 1);
        a.g = nullptr;
        a.tab = pl->tab_dev(t);
        a.l1 = pl->l1_dev(t);
        a.sigma = 2.0 * p2[j];
        a.out = O0;
        a.out_mode = 0;
        FPS_HIP(timed_sweep(pl, a, st));
        FPS_HIP(fps::launch_reduce(lv, pl->ctab_dev(t), ab, -a.sigma, npad, a.nc0, a.nc1, L.ncmax,
                                   st, (int)npad, S.lvb, S.abb));
        fps::SweepArgs b = a;
        b.in = O0;
        b.ab_prev = ab;
        b.tab_prev = pl->tab_dev(t);
        b.g = RX;
        b.sg = -1.0;
        b.og = 0.0;
        b.sigma = last ? 0.0 : p2[j] + p2[j + 1];
        b.out = O1;
        b.out_mode = last ? 1 : 0;
        FPS_HIP(timed_sweep(pl, b, st));
        FPS_HIP(fps::launch_reduce(lv, pl->ctab_dev(t), ab, last ? 1.0 : -b.sigma, npad, b.nc0,
                                   b.nc1, L.ncmax, st, (int)npad, S.lvb, S.abb));
      }
    }
    if (pl->nlds) continue;  // the inner launch wrote zR
    const double *tl = pl->tab_dev(t0 + J2 - 1);
    if (i + 1 < J1) {
      FPS_HIP(fps::launch_cube_ifinal(O1, ab, tl, RX, B, ZR, p1[i + 1] - q1[i], 1.0, -1.0, npad,
                                      mp0, L.mstride, L.ncmax, st));
    } else {
      FPS_HIP(fps::launch_cube_ifinal(O1, ab, tl, nullptr, nullptr, ZR, 1.0, 0.0, 0.0, npad, mp0,
                                      L.mstride, L.ncmax, st));
    }
  }

  // Output: Y is in ZR.
  if (pl->out_basis == FPS_OUT_NATIVE) {
    FPS_HIP(fps::launch_permute3_out(ZR, U, L.n, npad, mp0, (const double *)pl->d_sinv.p, st));
    return FPS_OK;
  }
  const int64_t mq = pl->mqc[0] + pl->mqc[1], mb0 = pl->mqc[0];
  const double *MA[2] = {(const double *)pl->d_PA[0].p, (const double *)pl->d_PA[1].p};
  const double *MB[2] = {(const double *)pl->d_PB[0].p, (const double *)pl->d_PB[1].p};
  const int64_t ldb[2] = {pl->mop[0], pl->mop[1]};
  const int64_t N[2] = {L.m[0] > 0 ? L.mo[0] : 0, L.m[1] > 0 ? L.mo[1] : 0};
  const Dims d1{{npad, npad, mq}, {mp0, mp0, mb0}};
  const Dims d2{{npad, mq, mq}, {mp0, mb0, mb0}};
  const Dims d3{{mq, mq, mq}, {mb0, mb0, mb0}};
  std::vector<fps::GemmProb> px, pz;
  // An empty parity block (n = 1) leaves its output entries to no GEMM: clear
  // the temporaries first so that they read as zeros.
  const bool empty_block = L.m[0] == 0 || L.m[1] == 0;
  if (empty_block) FPS_HIP(fps::launch_fill(O0, npad * npad * mq, 0.0, st));
  mode_probs(ZR, full, O0, d1, 2, MA, ldm, MB, ldb, N, K, px);
  if ((s = launch_probs(px, st)) != FPS_OK) return s;
  if (empty_block) FPS_HIP(fps::launch_fill(RX, npad * mq * mq, 0.0, st));
  FPS_HIP(fps::launch_gemm_table((const fps::GemmDesc *)pl->d_gy_out.p,
                                 (const int *)pl->d_gy_map_out.p, pl->gy_tiles[1], w, nullptr, st));
  if (empty_block) FPS_HIP(fps::launch_fill(O0, mq * mq * mq, 0.0, st));
  mode_probs(RX, d2, O0, d3, 0, MA, ldm, MB, ldb, N, K, pz);
  if ((s = launch_probs(pz, st)) != FPS_OK) return s;
  FPS_HIP(fps::launch_permute3_out(O0, U, L.n + 2, mq, mb0, nullptr, st));
  return FPS_OK;
}

// --- z-eigenbasis method ---------------------------------------------------
//
// G^ = G x_z V^T (V: eigenvectors of A~, parity blocks), then on every slice
// c (eigenvalue mu_c, P = A~ + mu_c) Algorithm 2 for
//   A_s Z - Z B_s = F_s,  A_s = -mu^2 P^-1 (y, left), B_s = -P (x, right),
//   F_s = -G^_c,  Z = P Y_c,
// in pass form: R_0 = -F_s = G^_c;
//   x solve:  x = (P + p_j)^-1 R along x, out V - F = R - (p_j - q_j) x;
//   y solve:  x = (q_j P + mu^2)^-1 P V along y (stencil P), V = (V - F) - G^,
//             out R' = (V - F) - (q_j - p_{j+1}) x;
//   last y solve without the stencil: Y_c = -(q P + mu^2)^-1 V.
// Then Y = Y^ x_z V and the output map.

namespace {

void zeig_tables_of(const fps_plan *pl, int k, int j, int *t1, int *t2) {
  *t1 = pl->ztab0[k] + 2 * j;
  *t2 = pl->ztab0[k] + 2 * j + 1;
}

// Number of leading (longest) slices to iterate on a second stream.  Model
// of one stream running slices lo .. hi-1 alone: (its largest J) x a fixed
// cost per ADI step (four launches) + (its slice steps) x the HBM time of
// one slice step (40 bytes per dof).  The leading group grows while its
// time stays within 0.85 of the rest's: the long slices' sparse launches
// at the end then run beside the bulk, while both streams, which share HBM,
// stay unequal enough that the caller's stream sets the pace (n = 256:
// 78 of 256 slices; measured 5.65 ms per solve against 6.07 on one stream,
// 5.91 with 128 and 6.15 with 196 leading slices).  Latency-bound runs
// (small n) keep one stream.
int zeig_split(const std::vector<int> &J, int64_t npad, double bytes_per_dof = 40.0) {
  const int K = (int)J.size();
  const double lat = 17.0;                                                        // us per step
  const double b = bytes_per_dof * (double)npad * (double)npad / 5.6e12 * 1e6;  // us per slice step
  double tot = 0.0, lead = 0.0;
  for (int k = 0; k < K; ++k) tot += J[k];
  int nl = 0;
  for (int k = 1; k < K; ++k) {  // J is descending: slices 0 .. k-1 lead
    lead += J[k - 1];
    if (J[0] * lat + lead * b <= 0.85 * (J[k] * lat + (tot - lead) * b)) nl = k;
  }
  return nl;
}

}  // namespace

fps_status zeig_common(fps_plan *pl);

// Refined plans: the schedule of refinement rounds, and per round and slice
// the shifts of the K-form slice equation
//   (|mu| K + 1/2) dY + dY (|mu| K + 1/2) = K q K,   K = -A~^-1,
// (multiply A~ dY A~ + mu (A~ dY + dY A~) = -q by K on both sides; K A~ = -I,
// mu < 0).  sigma(|mu| K + 1/2) lies in [|mu| / |ea| + 1/2, |mu| / |eb| + 1/2]
// for sigma(A~) in [ea, eb], so Algorithm 2 runs in the square's symmetric
// pass form with -(|mu| K + 1/2) in place of A~, its shifts p in
// [-b, -a] applied by increasing |p|.  The shifted solve is
// (-(|mu| K + 1/2) + p)^-1 = (|mu| - s A~)^-1 A~ with s = 1/2 - p: the A~
// stencil, then a tridiagonal solve with the table of (p - 1/2) A~ + |mu|.
// Every sweep array stores in float: in this form a round contracts the
// error by ~1e-5 (emulated at n = 32 .. 256; the slice equations' own form
// (-mu^2 P^-1) Z - Z (-P) contracts by only 1e-2 .. 1e-4 per round with float
// storage, worse as n grows).
fps_status zeigr_build(fps_plan *pl, const std::vector<long double> lam[2], double ea, double eb) {
  const fps::Layout &L = pl->L;
  struct S {
    int slice;
    double mu;
  };
  std::vector<S> sl;
  for (int sp = 0; sp < 2; ++sp)
    for (int64_t k = 0; k < L.m[sp]; ++k)
      sl.push_back(S{(int)(sp * L.mp[0] + k), (double)lam[sp][(size_t)k]});
  // |mu| descending: J of every round is then non-increasing along the order
  std::stable_sort(sl.begin(), sl.end(),
                   [](const S &u, const S &v) { return std::fabs(u.mu) > std::fabs(v.mu); });
  const int K = (int)sl.size();
  const std::vector<RefineRound> sched = refine_schedule(pl->tol, false);
  pl->rounds = (int)sched.size();
  pl->rtol.clear();
  pl->rf32.clear();
  for (const RefineRound &r : sched) {
    pl->rtol.push_back(r.tol);
    pl->rf32.push_back(1);
  }
  pl->zrslice.resize(K);
  pl->zrmu_slice.assign((size_t)L.npad, 0.0);
  for (int k = 0; k < K; ++k) {
    pl->zrslice[k] = sl[k].slice;
    pl->zrmu_slice[(size_t)sl[k].slice] = sl[k].mu;
  }
  pl->zrJ.assign(pl->rounds, std::vector<int>(K, 0));
  pl->zrtab0.assign(pl->rounds, std::vector<int>(K, 0));
  pl->zractive.assign(pl->rounds, std::vector<int>());
  pl->zrJmax.assign(pl->rounds, 0);
  pl->zrrow0.assign(pl->rounds, 0);
  std::vector<double> alpha{1.0}, beta{0.0};  // table 0: A~
  pl->zp.assign(1, 0.0);                       // shift of each table (by table id)
  std::string err;
  pl->n_f32 = 0;
  for (int r = 0; r < pl->rounds; ++r) {
    for (int k = 0; k < K; ++k) {
      const double am = std::fabs(sl[k].mu);
      const double a = am / std::fabs(ea) + 0.5, b = am / std::fabs(eb) + 0.5;
      fps::ShiftSet sh;
      if (!fps::zolotarev_shifts(-b, -a, a, b, pl->rtol[(size_t)r], sh, err))
        return fail(FPS_E_ARG, err);
      std::reverse(sh.p.begin(), sh.p.end());  // increasing |p|
      std::reverse(sh.q.begin(), sh.q.end());
      if (r == 0 && k == 0) pl->shifts = sh;
      pl->zrJ[(size_t)r][(size_t)k] = sh.J;
      pl->zrtab0[(size_t)r][(size_t)k] = (int)alpha.size();
      for (int j = 0; j < sh.J; ++j) {
        alpha.push_back(sh.p[j] - 0.5);
        beta.push_back(am);
        pl->zp.push_back(sh.p[j]);
      }
      if (k > 0 && sh.J > pl->zrJ[(size_t)r][(size_t)k - 1])
        return fail(FPS_E_STATE, "internal: refined slice steps not sorted");
    }
    const int Jm = K > 0 ? pl->zrJ[(size_t)r][0] : 0;
    pl->zrJmax[(size_t)r] = Jm;
    pl->zractive[(size_t)r].assign((size_t)Jm, 0);
    for (int j = 0; j < Jm; ++j)
      for (int k = 0; k < K; ++k)
        if (pl->zrJ[(size_t)r][(size_t)k] > j) pl->zractive[(size_t)r][(size_t)j] = k + 1;
    if (r > 0) pl->zrrow0[(size_t)r] = pl->zrrow0[(size_t)r - 1] + pl->zrJmax[(size_t)r - 1];
    pl->n_f32 += Jm;
  }
  // the slice-count query reports round 0
  pl->zslice = pl->zrslice;
  pl->zJ = K > 0 ? pl->zrJ[0] : std::vector<int>();
  pl->zJmax = K > 0 ? pl->zrJmax[0] : 0;
  pl->zsplit = 0;
  // every round splits its longest slices off like the FP64 plan (float
  // storage: 8 + 12 bytes per dof and step)
  pl->zrsplit.assign((size_t)pl->rounds, 0);
  for (int r = 0; r < pl->rounds; ++r)
    pl->zrsplit[(size_t)r] = zeig_split(pl->zrJ[(size_t)r], L.npad, 20.0);
  fps::build_sweep_tables_ab(L, alpha, beta, pl->tab, pl->ctab, nullptr, pl->l1);
  return FPS_OK;
}

fps_status zeig_build(fps_plan *pl) {
  const int64_t n = pl->n;
  pl->zeig = true;
  pl->L = fps::make_layout(n);
  const fps::Layout &L = pl->L;
  const double delta = 1.0 / (30.0 * (double)n * (double)n * (double)n * (double)n);
  double ea = -1.0, eb = -delta;
  if (pl->flags & FPS_PLAN_TIGHT_SPECTRUM) spectrum_tight(n, &ea, &eb);
  // eigen-decomposition of the parity blocks of A~
  std::vector<long double> lam[2];
  for (int sp = 0; sp < 2; ++sp) {
    const int64_t m = L.m[sp];
    pl->zV[sp].assign((size_t)(m * m), 0.0);
    if (m == 0) continue;
    std::vector<long double> d(m), e(m > 1 ? m - 1 : 0), Q;
    for (int64_t k = 0; k < m; ++k) d[k] = fps::atilde_diag(2 * k + sp);
    for (int64_t k = 0; k + 1 < m; ++k) e[k] = fps::atilde_off(2 * k + sp);
    if (!fps::tridiag_eigen(d, e, Q)) return fail(FPS_E_STATE, "eigen-decomposition of A~ failed");
    lam[sp] = d;
    for (int64_t i = 0; i < m * m; ++i) pl->zV[sp][(size_t)i] = (double)Q[(size_t)i];
  }
  if (pl->prec == FPS_FP32_REFINED) {
    fps_status s = zeigr_build(pl, lam, ea, eb);
    if (s != FPS_OK) return s;
    return zeig_common(pl);
  }
  // per-slice shifts
  struct Slice {
    int slice, J;
    double mu;
    fps::ShiftSet sh;
  };
  std::vector<Slice> sl;
  std::string err;
  for (int sp = 0; sp < 2; ++sp)
    for (int64_t k = 0; k < L.m[sp]; ++k) {
      Slice x;
      x.slice = (int)(sp * L.mp[0] + k);
      x.mu = (double)lam[sp][(size_t)k];
      const double am = std::fabs(x.mu);
      const double a = x.mu * x.mu / (std::fabs(ea) + am), b = x.mu * x.mu / (std::fabs(eb) + am);
      const double c = std::fabs(eb) + am, d = std::fabs(ea) + am;
      if (!fps::zolotarev_shifts(a, b, c, d, pl->tol, x.sh, err)) return fail(FPS_E_ARG, err);
      x.J = x.sh.J;
      sl.push_back(x);
    }
  std::stable_sort(sl.begin(), sl.end(), [](const Slice &u, const Slice &v) { return u.J > v.J; });
  const int K = (int)sl.size();
  pl->zslice.resize(K);
  pl->zJ.resize(K);
  pl->zmu.resize(K);
  pl->ztab0.resize(K);
  pl->zJmax = K > 0 ? sl[0].J : 0;
  pl->zp.clear();
  pl->zq.clear();
  std::vector<double> alpha, beta;
  for (int k = 0; k < K; ++k) {
    pl->zslice[k] = sl[k].slice;
    pl->zJ[k] = sl[k].J;
    pl->zmu[k] = sl[k].mu;
    pl->ztab0[k] = (int)alpha.size();
    const double mu = sl[k].mu;
    for (int j = 0; j < sl[k].J; ++j) {
      pl->zp.push_back(sl[k].sh.p[j]);
      pl->zq.push_back(sl[k].sh.q[j]);
      alpha.push_back(1.0);  // x solve: A~ + (mu + p)
      beta.push_back(mu + sl[k].sh.p[j]);
      alpha.push_back(sl[k].sh.q[j]);  // y solve: q A~ + (mu^2 + q mu)
      beta.push_back(mu * mu + sl[k].sh.q[j] * mu);
    }
  }
  pl->zactive.assign(pl->zJmax + 1, 0);
  for (int j = 0; j <= pl->zJmax; ++j)
    for (int k = 0; k < K; ++k)
      if (pl->zJ[k] > j) pl->zactive[j] = k + 1;
  pl->zsplit = zeig_split(pl->zJ, L.npad);
  // report the largest slice iteration as the plan's J and its shifts
  pl->shifts = K > 0 ? sl[0].sh : fps::ShiftSet{};
  fps::build_sweep_tables_ab(L, alpha, beta, pl->tab, pl->ctab, nullptr, pl->l1);
  return zeig_common(pl);
}

// Maps, stencil and workspace layout shared by the FP64 and refined
// z-eigenbasis plans.
fps_status zeig_common(fps_plan *pl) {
  const int64_t n = pl->n;
  const fps::Layout &L = pl->L;
  fps::build_conversions(L, pl->Rs, pl->P);
  for (int s2 = 0; s2 < 2; ++s2) {
    pl->mop[s2] = (L.mo[s2] + fps::kPad - 1) / fps::kPad * fps::kPad;
    pl->mqc[s2] = (L.mo[s2] + 1) / 2 * 2;
  }
  pl->sinv.resize(n);
  for (int64_t i = 0; i < n; ++i) pl->sinv[i] = 1.0 / std::sqrt((double)(i + 1) * (double)(i + 2));
  pl->sdiag.assign(L.npad, 0.0);
  pl->soff.assign(L.npad, 0.0);
  for (int sp = 0; sp < 2; ++sp)
    for (int64_t k = 0; k < L.m[sp]; ++k) {
      const int64_t r = sp * L.mp[0] + k, i = 2 * k + sp;
      pl->sdiag[r] = fps::atilde_diag(i);
      if (k + 1 < L.m[sp]) pl->soff[r] = fps::atilde_off(i);
    }
  const int64_t vol = align256(L.npad * L.npad * L.npad * 8);
  const int64_t ch = L.npad * L.npad;
  pl->off_G = 0;      // G^ (eigen-z slices, [c][y][x])
  pl->off_ZR = vol;   // Y^
  pl->off_RX = 2 * vol;
  pl->off_RXT = 3 * vol;  // refined plans: transposed float slice arrays
  pl->off_O0 = 4 * vol;
  pl->off_O1 = 5 * vol;
  pl->off_lv = 6 * vol;
  pl->off_lv2 = pl->off_lv + align256(L.ncmax * 4 * ch * 8);
  pl->zfused = L.ncmax <= 2;
  pl->off_ab = pl->off_lv2 + (pl->zfused ? align256(L.ncmax * 4 * ch * 8) : 0);
  pl->ws_bytes = pl->off_ab + align256(2 * L.ncmax * ch * 2 * 8);
  const int64_t mq = pl->mqc[0] + pl->mqc[1];
  if (L.npad * L.npad * mq * 8 > 2 * vol || mq * mq * mq * 8 > 2 * vol ||
      L.npad * mq * mq * 8 > 2 * vol)
    return fail(FPS_E_STATE, "internal: cube output temporaries exceed the workspace");
  return FPS_OK;
}

// The plan's default-priority side stream and its fork / join events
// (z-eigenbasis plans that split their slices over two streams; 2-D plans
// that split their ADI by row parity).
fps_status create_side_stream(fps_plan *pl) {
  if (pl->zside != nullptr) return FPS_OK;
  if (hipStreamCreateWithFlags(&pl->zside, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&pl->zfork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&pl->zjoin, hipEventDisableTiming) != hipSuccess) {
    if (pl->zside) (void)hipStreamDestroy(pl->zside);
    if (pl->zfork) (void)hipEventDestroy(pl->zfork);
    if (pl->zjoin) (void)hipEventDestroy(pl->zjoin);
    pl->zside = nullptr;
    pl->zfork = pl->zjoin = nullptr;
    return fail(FPS_E_HIP, "creating the slice side stream failed");
  }
  return FPS_OK;
}

// Refined plans: per-slice mu (residual kernel), and the sweep and carry
// descriptors of every round, [row][half][sorted slice] with row =
// zrrow0[r] + j (see zeigr_build for the pass form).
fps_status zeigr_upload(fps_plan *pl) {
  const fps::Layout &L = pl->L;
  const int64_t npad = L.npad, ch = npad * npad;
  const int K = (int)pl->zrslice.size();
  fps_status s;
  const int nbx_s = (int)(npad / fps::kCols), nch = (int)(L.nc[0] + L.nc[1]);
  const int nsw = nbx_s * nch;
  const int rchains = fps::reduce_chains(L.ncmax);
  const int nbx_r = (int)((npad + rchains - 1) / rchains);
  const int nrd = nbx_r * 2;
  const int64_t lvb = L.ncmax * 4 * npad, abb = 2 * L.ncmax * npad * 2;  // doubles per slice
  const int rows = pl->zrrow0.back() + pl->zrJmax.back();
  const size_t Kc = (size_t)(K > 0 ? K : 1);
  std::vector<fps::BatchSweep> sw((size_t)rows * 2 * Kc);
  std::vector<fps::BatchReduce> rd((size_t)rows * 2 * Kc);
  std::vector<const double *> fin((size_t)pl->rounds * npad, nullptr);
  const double *pre_d = (const double *)pl->d_pre.p;
  const bool fused = pl->zfused;
  std::vector<fps::BatchReduce> rdfin((size_t)pl->rounds * Kc);
  for (int k = 0; k < K; ++k) {
    const int64_t c = pl->zrslice[k];
    const int64_t so = c * ch * 4;  // the float arrays hold slices at a stride of npad^2 floats
    const int64_t lvo = pl->off_lv + c * lvb * 8, abo = pl->off_ab + c * abb * 8;
    const int64_t lvo2 = fused ? pl->off_lv2 + c * lvb * 8 : lvo;
    fps::SweepArgs A{};
    A.npad = npad;
    A.ncols = npad;
    A.ld = npad;
    A.nbatch = 1;
    A.mp0 = L.mp[0];
    A.mp1 = L.mp[1];
    A.mstride = L.mstride;
    A.ncmax = L.ncmax;
    A.nc0 = (int)L.nc[0];
    A.nc1 = (int)L.nc[1];
    A.lv = (double *)(intptr_t)lvo;
    A.pre = pre_d;
    A.pre_shift = 0.0;
    A.in_f32 = A.out_f32 = 1;
    for (int r = 0; r < pl->rounds; ++r) {
      const int J = pl->zrJ[(size_t)r][(size_t)k], t0 = pl->zrtab0[(size_t)r][(size_t)k];
      for (int j = 0; j < J; ++j) {
        const int t = t0 + j;
        const bool last = j == J - 1;
        const double pj = pl->zp[(size_t)t], pn = last ? 0.0 : pl->zp[(size_t)t + 1];
        fps::SweepArgs a1 = A;
        a1.in = (const void *)(intptr_t)((j == 0 ? pl->off_RXT : pl->off_O1) + so);
        a1.in_scale = j == 0 ? -1.0 : 1.0;
        a1.ab_prev = j == 0 ? nullptr : (const double *)(intptr_t)abo;
        a1.tab_prev = j == 0 ? nullptr : pl->tab_dev(t - 1);
        a1.g = nullptr;
        a1.tab = pl->tab_dev(t);
        a1.l1 = pl->l1_dev(t);
        a1.sigma = 2.0 * pj;
        a1.out = (void *)(intptr_t)(pl->off_O0 + so);
        a1.out_mode = 0;
        fps::SweepArgs a2 = a1;
        a2.in = (const void *)(intptr_t)(pl->off_O0 + so);
        a2.in_scale = 1.0;
        a2.ab_prev = (const double *)(intptr_t)abo;
        a2.tab_prev = pl->tab_dev(t);
        a2.g = (const void *)(intptr_t)(pl->off_RX + so);
        a2.g_f32 = 1;
        a2.sg = 1.0;
        a2.og = 0.0;
        a2.sigma = last ? 0.0 : pj + pn;
        a2.out = (void *)(intptr_t)(pl->off_O1 + so);
        a2.out_mode = last ? 1 : 0;
        if (fused) {  // carries from the producer's boundary values, no carry launch
          a2.lv = (double *)(intptr_t)lvo2;
          if (j > 0) {
            a1.ab_prev = nullptr;
            a1.lv_prev = (const double *)(intptr_t)lvo2;
            a1.ctab_prev = pl->ctab_dev(t - 1);
            a1.carry_scale = -(pl->zp[(size_t)t - 1] + pj);  // the previous second half-step
          }
          a2.ab_prev = nullptr;
          a2.lv_prev = (const double *)(intptr_t)lvo;
          a2.ctab_prev = pl->ctab_dev(t);
          a2.carry_scale = -a1.sigma;
          if (last)
            rdfin[(size_t)r * Kc + k] =
                fps::BatchReduce{lvo2, abo, pl->ctab_dev(t), 1.0, npad, L.ncmax, (int)L.nc[0],
                                 (int)L.nc[1], k * nrd, nbx_r};
        }
        const size_t row = (size_t)pl->zrrow0[(size_t)r] + (size_t)j;
        const size_t i1 = (row * 2 + 0) * Kc + k, i2 = (row * 2 + 1) * Kc + k;
        sw[i1] = fps::BatchSweep{a1, k * nsw, nbx_s};
        sw[i2] = fps::BatchSweep{a2, k * nsw, nbx_s};
        rd[i1] = fps::BatchReduce{lvo, abo, pl->ctab_dev(t), -a1.sigma, npad, L.ncmax,
                                  (int)L.nc[0], (int)L.nc[1], k * nrd, nbx_r};
        rd[i2] = fps::BatchReduce{lvo, abo, pl->ctab_dev(t), last ? 1.0 : -a2.sigma, npad,
                                  L.ncmax, (int)L.nc[0], (int)L.nc[1], k * nrd, nbx_r};
      }
      fin[(size_t)r * npad + c] = J > 0 ? pl->tab_dev(t0 + J - 1) : nullptr;
    }
  }
  std::vector<int> swmap((size_t)K * nsw), rdmap((size_t)K * nrd);
  for (int k = 0; k < K; ++k) {
    std::fill(swmap.begin() + (size_t)k * nsw, swmap.begin() + (size_t)(k + 1) * nsw, k);
    std::fill(rdmap.begin() + (size_t)k * nrd, rdmap.begin() + (size_t)(k + 1) * nrd, k);
  }
  pl->zsw_start.assign(1, nsw);
  pl->zrd_start.assign(1, nrd);
  if ((s = upload(pl->d_zrsw, sw)) != FPS_OK || (s = upload(pl->d_zrrd, rd)) != FPS_OK ||
      (s = upload(pl->d_zswmap, swmap)) != FPS_OK || (s = upload(pl->d_zrdmap, rdmap)) != FPS_OK ||
      (s = upload(pl->d_zrfin, fin)) != FPS_OK || (s = upload(pl->d_zmu, pl->zrmu_slice)) != FPS_OK ||
      (fused && (s = upload(pl->d_zrdfin, rdfin)) != FPS_OK))
    return s;
  for (int sp : pl->zrsplit)
    if (sp > 0) return create_side_stream(pl);
  return FPS_OK;
}

fps_status zeig_upload(fps_plan *pl) {
  const fps::Layout &L = pl->L;
  const int64_t npad = L.npad, ch = npad * npad;
  fps_status s;
  // dense map blocks (zero padded): Rs (x, y input), V^T Rs (z input), P (x, y
  // output), P V (z output), V (z back-transform for native output)
  std::vector<double> RsA[2], RsB[2], Mz[2], PA[2], PB[2], PV[2], Vz[2];
  for (int sp = 0; sp < 2; ++sp) {
    const int64_t m = L.m[sp], mp = L.mp[sp], mo = L.mo[sp], mop = pl->mop[sp];
    RsA[sp].assign((size_t)(mp * mp), 0.0);
    RsB[sp].assign((size_t)(mp * mp), 0.0);
    Mz[sp].assign((size_t)(mp * mp), 0.0);
    Vz[sp].assign((size_t)(mp * mp), 0.0);
    PA[sp].assign((size_t)(mop * mp), 0.0);
    PB[sp].assign((size_t)(mp * mop), 0.0);
    PV[sp].assign((size_t)(mop * mp), 0.0);
    const std::vector<double> &V = pl->zV[sp];  // V[i][k]: component i of eigenvector k
    for (int64_t i = 0; i < m; ++i)
      for (int64_t k = 0; k < m; ++k) {
        RsA[sp][(size_t)(i * mp + k)] = pl->Rs[sp][(size_t)(i * m + k)];
        RsB[sp][(size_t)(k * mp + i)] = pl->Rs[sp][(size_t)(i * m + k)];
        Vz[sp][(size_t)(i * mp + k)] = V[(size_t)(i * m + k)];
      }
    for (int64_t k = 0; k < m; ++k)  // (V^T Rs)[k][b] = sum_i V[i][k] Rs[i][b]
      for (int64_t b = 0; b < m; ++b) {
        long double acc = 0.0L;
        for (int64_t i = 0; i < m; ++i)
          acc += (long double)V[(size_t)(i * m + k)] * pl->Rs[sp][(size_t)(i * m + b)];
        Mz[sp][(size_t)(k * mp + b)] = (double)acc;
      }
    for (int64_t i = 0; i < mo; ++i) {
      for (int64_t k = 0; k < m; ++k) {
        PA[sp][(size_t)(i * mp + k)] = pl->P[sp][(size_t)(i * m + k)];
        PB[sp][(size_t)(k * mop + i)] = pl->P[sp][(size_t)(i * m + k)];
      }
      for (int64_t k = 0; k < m; ++k) {  // (P V)[i][k]
        long double acc = 0.0L;
        for (int64_t b = 0; b < m; ++b)
          acc += (long double)pl->P[sp][(size_t)(i * m + b)] * V[(size_t)(b * m + k)];
        PV[sp][(size_t)(i * mp + k)] = (double)acc;
      }
    }
  }
  // the stencil A~ (diagonal, coupling), then the identity stencil (ones,
  // zeros) that the y solves of slices at their last step take, so that they
  // run in the same launch as the stencil y solves of the others
  std::vector<double> pre(pl->sdiag);
  pre.insert(pre.end(), pl->soff.begin(), pl->soff.end());
  pre.insert(pre.end(), (size_t)npad, 1.0);
  pre.insert(pre.end(), (size_t)npad, 0.0);
  if ((s = upload(pl->d_tab, pl->tab)) != FPS_OK || (s = upload(pl->d_ctab, pl->ctab)) != FPS_OK ||
      (s = upload(pl->d_l1, pl->l1)) != FPS_OK || (s = upload(pl->d_sinv, pl->sinv)) != FPS_OK ||
      (s = upload(pl->d_pre, pre)) != FPS_OK)
    return s;
  for (int sp = 0; sp < 2; ++sp)
    if ((s = upload(pl->d_RsA[sp], RsA[sp])) != FPS_OK ||
        (s = upload(pl->d_RsB[sp], RsB[sp])) != FPS_OK || (s = upload(pl->d_Mz[sp], Mz[sp])) != FPS_OK ||
        (s = upload(pl->d_PA[sp], PA[sp])) != FPS_OK || (s = upload(pl->d_PB[sp], PB[sp])) != FPS_OK ||
        (s = upload(pl->d_PV[sp], PV[sp])) != FPS_OK || (s = upload(pl->d_Vz[sp], Vz[sp])) != FPS_OK)
      return s;
  // mode-y GEMM tables (input: Rs; output: P)
  const Dims full = full_dims(L);
  const int64_t K2[2] = {L.mp[0], L.mp[1]};
  const int64_t lda[2] = {L.mp[0], L.mp[1]};
  {
    const double *MA[2] = {(const double *)pl->d_RsA[0].p, (const double *)pl->d_RsA[1].p};
    const int64_t N[2] = {L.m[0] > 0 ? L.mp[0] : 0, L.m[1] > 0 ? L.mp[1] : 0};
    std::vector<fps::GemmProb> probs;
    mode_probs((const double *)(intptr_t)pl->off_O1, full, (double *)(intptr_t)pl->off_O0, full, 1,
               MA, lda, nullptr, lda, N, K2, probs);
    if ((s = upload_table(probs, pl->d_gy_in, pl->d_gy_map_in, pl->gy_tiles[0])) != FPS_OK) return s;
  }
  {
    const int64_t mq = pl->mqc[0] + pl->mqc[1];
    const Dims di{{L.npad, L.npad, mq}, {L.mp[0], L.mp[0], pl->mqc[0]}};
    const Dims dout{{L.npad, mq, mq}, {L.mp[0], pl->mqc[0], pl->mqc[0]}};
    const double *MA[2] = {(const double *)pl->d_PA[0].p, (const double *)pl->d_PA[1].p};
    const int64_t N[2] = {L.m[0] > 0 ? L.mo[0] : 0, L.m[1] > 0 ? L.mo[1] : 0};
    std::vector<fps::GemmProb> probs;
    mode_probs((const double *)(intptr_t)pl->off_O0, di, (double *)(intptr_t)pl->off_RX, dout, 1,
               MA, lda, nullptr, lda, N, K2, probs);
    if ((s = upload_table(probs, pl->d_gy_out, pl->d_gy_map_out, pl->gy_tiles[1])) != FPS_OK)
      return s;
  }
  if (pl->prec == FPS_FP32_REFINED) return zeigr_upload(pl);
  // per-slice sweep and carry descriptors: [step][half][sorted slice]
  const int K = (int)pl->zslice.size(), J = pl->zJmax;
  const int nbx_s = (int)(npad / fps::kCols), nch = (int)(L.nc[0] + L.nc[1]);
  const int nsw = nbx_s * nch;
  const int rchains = fps::reduce_chains(L.ncmax);  // as launch_reduce_batch(ncmax_max = L.ncmax)
  const int nbx_r = (int)((npad + rchains - 1) / rchains);
  const int nrd = nbx_r * 2;
  const int64_t lvb = L.ncmax * 4 * npad, abb = 2 * L.ncmax * npad * 2;  // doubles per slice
  std::vector<fps::BatchSweep> sw((size_t)J * 2 * (K > 0 ? K : 1));
  std::vector<fps::BatchReduce> rd((size_t)J * 2 * (K > 0 ? K : 1));
  const double *pre_d = (const double *)pl->d_pre.p;
  const bool fused = pl->zfused;
  std::vector<fps::BatchReduce> rdfin((size_t)(K > 0 ? K : 1));
  for (int k = 0; k < K; ++k) {
    const int64_t c = pl->zslice[k];
    const int64_t so = c * ch * 8;  // slice byte offset in an npad^3 array
    const int64_t lvo = pl->off_lv + c * lvb * 8, abo = pl->off_ab + c * abb * 8;
    const int64_t lvo2 = fused ? pl->off_lv2 + c * lvb * 8 : lvo;
    double sigma2_prev = 0.0;  // the second half-step's sigma of the previous step
    fps::SweepArgs A{};
    A.npad = npad;
    A.ncols = npad;
    A.ld = npad;
    A.nbatch = 1;
    A.mp0 = L.mp[0];
    A.mp1 = L.mp[1];
    A.mstride = L.mstride;
    A.ncmax = L.ncmax;
    A.nc0 = (int)L.nc[0];
    A.nc1 = (int)L.nc[1];
    A.lv = (double *)(intptr_t)lvo;
    const double mu = pl->zmu[k];
    for (int j = 0; j < pl->zJ[k]; ++j) {
      int t1, t2;
      zeig_tables_of(pl, k, j, &t1, &t2);
      const bool last = j == pl->zJ[k] - 1;
      const double pj = pl->zp[(size_t)t1 / 2], qj = pl->zq[(size_t)t1 / 2];
      const double pn = last ? 0.0 : pl->zp[(size_t)t1 / 2 + 1];
      // Every slice array keeps G^'s layout ([y][x]): the x solve runs along
      // the storage rows (batched row-chain sweep, out_mode 0: the row-wise
      // store of v - sigma x), the y solve along the storage columns, stored
      // in place (out_mode 2; 1 at the last step).
      fps::SweepArgs a1 = A;
      a1.in = (const void *)(intptr_t)((j == 0 ? pl->off_G : pl->off_O1) + so);
      a1.in_scale = 1.0;
      a1.ab_prev = j == 0 ? nullptr : (const double *)(intptr_t)abo;
      a1.tab_prev = j == 0 ? nullptr : pl->tab_dev(t1 - 1);
      a1.g = nullptr;
      a1.tab = pl->tab_dev(t1);
      a1.l1 = pl->l1_dev(t1);
      a1.sigma = pj - qj;
      a1.out = (void *)(intptr_t)(pl->off_O0 + so);
      a1.out_mode = 0;
      fps::SweepArgs a2 = A;
      a2.in = (const void *)(intptr_t)(pl->off_O0 + so);
      a2.in_scale = 1.0;
      a2.ab_prev = (const double *)(intptr_t)abo;
      a2.tab_prev = pl->tab_dev(t1);
      a2.g = (const void *)(intptr_t)(pl->off_G + so);
      a2.sg = -1.0;
      a2.og = 0.0;
      // last step: the identity stencil (P = I: the plain y solve, exactly)
      a2.pre = last ? pre_d + 2 * npad : pre_d;
      a2.pre_shift = last ? 0.0 : mu;
      a2.tab = pl->tab_dev(t2);
      a2.l1 = pl->l1_dev(t2);
      a2.sigma = last ? 0.0 : qj - pn;
      a2.out = (void *)(intptr_t)(pl->off_O1 + so);
      a2.out_mode = last ? 1 : 2;
      if (fused) {  // carries from the producer's boundary values, no carry launch
        a2.lv = (double *)(intptr_t)lvo2;
        if (j > 0) {
          a1.ab_prev = nullptr;
          a1.lv_prev = (const double *)(intptr_t)lvo2;
          a1.ctab_prev = pl->ctab_dev(t1 - 1);
          a1.carry_scale = -sigma2_prev;
        }
        a2.ab_prev = nullptr;
        a2.lv_prev = (const double *)(intptr_t)lvo;
        a2.ctab_prev = pl->ctab_dev(t1);
        a2.carry_scale = -a1.sigma;
        sigma2_prev = a2.sigma;
        if (last)
          rdfin[(size_t)k] = fps::BatchReduce{lvo2, abo, pl->ctab_dev(t2), 1.0, npad, L.ncmax,
                                              (int)L.nc[0], (int)L.nc[1], k * nrd, nbx_r};
      }
      const size_t i1 = ((size_t)j * 2 + 0) * K + k, i2 = ((size_t)j * 2 + 1) * K + k;
      sw[i1] = fps::BatchSweep{a1, k * nsw, nbx_s};
      sw[i2] = fps::BatchSweep{a2, k * nsw, nbx_s};
      rd[i1] = fps::BatchReduce{lvo, abo, pl->ctab_dev(t1), -a1.sigma, npad, L.ncmax,
                                (int)L.nc[0], (int)L.nc[1], k * nrd, nbx_r};
      rd[i2] = fps::BatchReduce{lvo, abo, pl->ctab_dev(t2), last ? 1.0 : -a2.sigma, npad, L.ncmax,
                                (int)L.nc[0], (int)L.nc[1], k * nrd, nbx_r};
    }
  }
  std::vector<int> swmap((size_t)(K * nsw)), rdmap((size_t)(K * nrd));
  for (int k = 0; k < K; ++k) {
    std::fill(swmap.begin() + (size_t)k * nsw, swmap.begin() + (size_t)(k + 1) * nsw, k);
    std::fill(rdmap.begin() + (size_t)k * nrd, rdmap.begin() + (size_t)(k + 1) * nrd, k);
  }
  std::vector<const double *> fin((size_t)npad, nullptr);
  for (int k = 0; k < K; ++k) {
    int t1, t2;
    zeig_tables_of(pl, k, pl->zJ[k] - 1, &t1, &t2);
    fin[(size_t)pl->zslice[k]] = pl->tab_dev(t2);
  }
  pl->zsw_start.assign(1, nsw);
  pl->zrd_start.assign(1, nrd);
  if ((s = upload(pl->d_zsw, sw)) != FPS_OK || (s = upload(pl->d_zrd, rd)) != FPS_OK ||
      (s = upload(pl->d_zswmap, swmap)) != FPS_OK || (s = upload(pl->d_zrdmap, rdmap)) != FPS_OK ||
      (s = upload(pl->d_zfin, fin)) != FPS_OK ||
      (fused && (s = upload(pl->d_zrdfin, rdfin)) != FPS_OK))
    return s;
  // The LDS-resident form: per sorted slice its storage slice, steps, first
  // table, mu and the sigmas of its steps (those of the descriptors above),
  // then every storage slice without steps.
  pl->zlds = fps::zeig_lds_fits(L.m[0], L.m[1]) && L.mp[0] <= 128 && npad - L.mp[0] <= 128 &&
             L.mstride % fps::kZeigLdsChunk == 0;
  if (pl->zlds) {
    std::vector<int> zs, zj, zt, zo;
    std::vector<double> zm, sg;
    std::vector<char> seen((size_t)npad, 0);
    for (int k = 0; k < K; ++k) {
      zs.push_back(pl->zslice[k]);
      zj.push_back(pl->zJ[k]);
      zt.push_back(pl->ztab0[k]);
      zo.push_back((int)sg.size());
      zm.push_back(pl->zmu[k]);
      seen[(size_t)pl->zslice[k]] = 1;
      for (int j = 0; j < pl->zJ[k]; ++j) {
        int t1, t2;
        zeig_tables_of(pl, k, j, &t1, &t2);
        const bool last = j == pl->zJ[k] - 1;
        const double pj = pl->zp[(size_t)t1 / 2], qj = pl->zq[(size_t)t1 / 2];
        const double pn = last ? 0.0 : pl->zp[(size_t)t1 / 2 + 1];
        sg.push_back(pj - qj);
        sg.push_back(last ? 0.0 : qj - pn);
      }
    }
    for (int64_t c = 0; c < npad; ++c)
      if (!seen[(size_t)c]) {
        zs.push_back((int)c);
        zj.push_back(0);
        zt.push_back(0);
        zo.push_back(0);
        zm.push_back(0.0);
      }
    if (sg.empty()) sg.push_back(0.0);
    std::vector<double> t32, c32;  // multipliers of the kernel's chunks
    fps::build_chunk_tables(L, pl->tab, fps::kZeigLdsChunk, t32, c32);
    if ((s = upload(pl->d_zl_slice, zs)) != FPS_OK || (s = upload(pl->d_zl_J, zj)) != FPS_OK ||
        (s = upload(pl->d_zl_tab0, zt)) != FPS_OK || (s = upload(pl->d_zl_sig0, zo)) != FPS_OK ||
        (s = upload(pl->d_zl_mu, zm)) != FPS_OK || (s = upload(pl->d_zl_sig, sg)) != FPS_OK ||
        (s = upload(pl->d_zl_tab32, t32)) != FPS_OK || (s = upload(pl->d_zl_ctab32, c32)) != FPS_OK)
      return s;
    return FPS_OK;  // one launch: no side stream
  }
  if (pl->zsplit > 0) return create_side_stream(pl);
  return FPS_OK;
}

// Refined plans: the rounds of Y^ <- Y^ + dY on every slice.  Round r: the
// negated residual q = G^ + A~ Y^ A~ + mu (A~ Y^ + Y^ A~) (FP64, stored in
// float, in O0); H = K q K = A~^-1 q A~^-1 by two shift-0 solves along the
// rows (the first stores x transposed, the second in place, so the second
// leaves H^T), its carries applied and H^T, H stored in float (RXT, RX);
// then the K-form Algorithm 2 of every slice in float (stencil passes on
// tables (p - 1/2) A~ + |mu|; step 0 reads -H^T, every second half-step adds
// H), and dY (float, carries pending) is added into Y^.
fps_status zeigr_adi(fps_plan *pl, char *w, hipStream_t st) {
  const fps::Layout &L = pl->L;
  const int64_t npad = L.npad, mp0 = L.mp[0];
  double *Gh = (double *)(w + pl->off_G), *Yh = (double *)(w + pl->off_ZR);
  float *q = (float *)(w + pl->off_O0), *x1 = (float *)(w + pl->off_O1);
  float *HT = (float *)(w + pl->off_RXT), *H = (float *)(w + pl->off_RX);
  double *lv = (double *)(w + pl->off_lv), *ab = (double *)(w + pl->off_ab);
  double *lv2 = (double *)(w + pl->off_lv2);
  const double *dv = (const double *)pl->d_pre.p, *ev = dv + npad;
  const int64_t lvb = L.ncmax * 4 * npad, abb = 2 * L.ncmax * npad * 2;
  const int K = (int)pl->zrslice.size();
  const size_t Kc = (size_t)(K > 0 ? K : 1);
  const int nsw = pl->zsw_start[0], nrd = pl->zrd_start[0];
  const fps::BatchSweep *dsw = (const fps::BatchSweep *)pl->d_zrsw.p;
  const fps::BatchReduce *drd = (const fps::BatchReduce *)pl->d_zrrd.p;
  const int *swmap = (const int *)pl->d_zswmap.p, *rdmap = (const int *)pl->d_zrdmap.p;
  const double *const *fin = (const double *const *)pl->d_zrfin.p;
  fps::SweepArgs t1{}, t2{};
  t1.pre = t2.pre = dv;
  t1.in_f32 = t1.out_f32 = 1;
  t2.in_f32 = t2.g_f32 = t2.out_f32 = 1;
  auto sweep = [&](const fps::SweepArgs &types, bool with_g, const fps::BatchSweep *d, int nwg,
                   int wg_base, hipStream_t s2) -> hipError_t {
    const bool t = pl->ev_used * 2 + 1 < (int64_t)pl->ev.size();
    const hipError_t e = fps::launch_sweep_batch(types, with_g, d, swmap, nwg, w, s2, wg_base,
                                                 t ? pl->ev[2 * pl->ev_used] : nullptr,
                                                 t ? pl->ev[2 * pl->ev_used + 1] : nullptr);
    if (t && e == hipSuccess) ++pl->ev_used;
    return e;
  };
  for (int r = 0; r < pl->rounds; ++r) {
    FPS_HIP(fps::launch_zeig_residual(Gh, r == 0 ? nullptr : Yh, dv, ev,
                                      (const double *)pl->d_zmu.p, q, npad, npad, st));
    // H = K q K on every slice (table 0 is A~): x = A~^-1 q stored
    // transposed, then A~^-1 x^T in place = H^T
    fps::SweepArgs S{};
    S.npad = npad;
    S.ncols = npad;
    S.ld = npad;
    S.nbatch = (int)npad;
    S.bstride = npad * npad;
    S.lvb = lvb;
    S.abb = abb;
    S.mp0 = L.mp[0];
    S.mp1 = L.mp[1];
    S.mstride = L.mstride;
    S.ncmax = L.ncmax;
    S.nc0 = (int)L.nc[0];
    S.nc1 = (int)L.nc[1];
    S.lv = lv;
    S.in = q;
    S.in_f32 = 1;
    S.in_scale = 1.0;
    S.tab = pl->tab_dev(0);
    S.l1 = pl->l1_dev(0);
    S.sigma = 0.0;
    S.out = x1;
    S.out_f32 = 1;
    S.out_mode = 3;
    FPS_HIP(fps::launch_sweep(S, st));
    S.in = x1;
    S.tab_prev = pl->tab_dev(0);
    if (pl->zfused) {  // the second solve forms the first one's carries itself
      S.lv_prev = lv;
      S.ctab_prev = pl->ctab_dev(0);
      S.carry_scale = 1.0;
      S.lv = lv2;
    } else {
      FPS_HIP(fps::launch_reduce(lv, pl->ctab_dev(0), ab, 1.0, npad, S.nc0, S.nc1, L.ncmax, st,
                                 (int)npad, lvb, abb));
      S.ab_prev = ab;
    }
    S.out = q;
    S.out_mode = 1;
    FPS_HIP(fps::launch_sweep(S, st));
    FPS_HIP(fps::launch_reduce(S.lv, pl->ctab_dev(0), ab, 1.0, npad, S.nc0, S.nc1, L.ncmax, st,
                               (int)npad, lvb, abb));
    FPS_HIP(fps::launch_slice_xfinal(q, ab, pl->tab_dev(0), HT, H, npad, mp0, L.mstride, L.ncmax,
                                     npad, st));
    // The K-form ADI of sorted slices lo .. hi-1 on stream s2: at step j
    // the active ones are lo .. min(zractive[r][j], hi) - 1 (J descending).
    auto run_group = [&](int lo, int hi, hipStream_t s2) -> hipError_t {
      hipError_t e = hipSuccess;
      for (int j = 0; j < pl->zrJmax[(size_t)r] && e == hipSuccess; ++j) {
        const int k1 = std::min(pl->zractive[(size_t)r][(size_t)j], hi);
        if (k1 <= lo) break;
        const size_t row = (size_t)pl->zrrow0[(size_t)r] + (size_t)j;
        const size_t o1 = (row * 2 + 0) * Kc, o2 = (row * 2 + 1) * Kc;
        e = sweep(t1, false, dsw + o1, (k1 - lo) * nsw, lo * nsw, s2);
        if (e == hipSuccess && !pl->zfused)
          e = fps::launch_reduce_batch(drd + o1, rdmap, (k1 - lo) * nrd, L.ncmax, w, s2, lo * nrd);
        if (e == hipSuccess) e = sweep(t2, true, dsw + o2, (k1 - lo) * nsw, lo * nsw, s2);
        if (e == hipSuccess && !pl->zfused)
          e = fps::launch_reduce_batch(drd + o2, rdmap, (k1 - lo) * nrd, L.ncmax, w, s2, lo * nrd);
      }
      return e;
    };
    // The round's longest slices iterate on the plan's side stream beside the
    // rest (as in the FP64 solve); per-dispatch timing keeps one stream.
    const int split = pl->zrsplit.empty() ? 0 : pl->zrsplit[(size_t)r];
    if (split > 0 && split < K && pl->zside && pl->ev.empty()) {
      std::lock_guard<std::mutex> lk(pl->zlock);
      FPS_HIP(hipEventRecord(pl->zfork, st));
      FPS_HIP(hipStreamWaitEvent(pl->zside, pl->zfork, 0));
      const hipError_t e1 = run_group(0, split, pl->zside);
      const hipError_t e2 = e1 == hipSuccess ? run_group(split, K, st) : hipSuccess;
      const hipError_t e3 = hipEventRecord(pl->zjoin, pl->zside);
      const hipError_t e4 = e3 == hipSuccess ? hipStreamWaitEvent(st, pl->zjoin, 0) : e3;
      FPS_HIP(e1);
      FPS_HIP(e2);
      FPS_HIP(e3);
      FPS_HIP(e4);
    } else {
      FPS_HIP(run_group(0, K, st));
    }
    if (pl->zfused)  // the carries of every slice's last half-step of the round
      FPS_HIP(fps::launch_reduce_batch((const fps::BatchReduce *)pl->d_zrdfin.p + (size_t)r * Kc,
                                       rdmap, K * nrd, L.ncmax, w, st));
    FPS_HIP(fps::launch_slice_final<float>(x1, ab, fin + (size_t)r * npad, Yh, 1.0, r > 0 ? 1 : 0,
                                           npad, mp0, L.mstride, L.ncmax, st));
  }
  return FPS_OK;
}

fps_status zeig_solve(fps_plan *pl, const double *F, double *U, char *w, hipStream_t st) {
  const fps::Layout &L = pl->L;
  const int64_t npad = L.npad, mp0 = L.mp[0];
  double *Gh = (double *)(w + pl->off_G);
  double *Yh = (double *)(w + pl->off_ZR), *RX = (double *)(w + pl->off_RX);
  double *O0 = (double *)(w + pl->off_O0), *O1 = (double *)(w + pl->off_O1);
  const Dims full = full_dims(L);
  const int64_t K2[2] = {L.mp[0], L.mp[1]};
  const int64_t ldm[2] = {L.mp[0], L.mp[1]};
  const int64_t Nfull[2] = {L.m[0] > 0 ? L.mp[0] : 0, L.m[1] > 0 ? L.mp[1] : 0};
  fps_status s;
  // Input map: G^ = F_T x_x Rs x_y Rs x_z (V^T Rs).
  FPS_HIP(fps::launch_permute3_in(F, O0, L.n, npad, mp0, st));
  {
    const double *MB[2] = {(const double *)pl->d_RsB[0].p, (const double *)pl->d_RsB[1].p};
    const double *MZ[2] = {(const double *)pl->d_Mz[0].p, (const double *)pl->d_Mz[1].p};
    std::vector<fps::GemmProb> px, pz;
    mode_probs(O0, full, O1, full, 2, MB, ldm, MB, ldm, Nfull, K2, px);
    if ((s = launch_probs(px, st)) != FPS_OK) return s;
    FPS_HIP(fps::launch_gemm_table((const fps::GemmDesc *)pl->d_gy_in.p,
                                   (const int *)pl->d_gy_map_in.p, pl->gy_tiles[0], w, nullptr, st));
    mode_probs(O0, full, Gh, full, 0, MZ, ldm, MZ, ldm, Nfull, K2, pz);
    if ((s = launch_probs(pz, st)) != FPS_OK) return s;
  }
  if (pl->prec == FPS_FP32_REFINED) {
    if ((s = zeigr_adi(pl, w, st)) != FPS_OK) return s;
  } else if (pl->zlds) {
    // Every slice's ADI in one launch, each parity block resident in one
    // workgroup's LDS (timed with the plan's first event pair, if any).
    fps::ZeigLdsArgs za{};
    za.G = Gh;
    za.Y = Yh;
    za.tab = (const double *)pl->d_tab.p;
    za.tab32 = (const double *)pl->d_zl_tab32.p;
    za.ctab32 = (const double *)pl->d_zl_ctab32.p;
    za.pre = (const double *)pl->d_pre.p;
    za.mu = (const double *)pl->d_zl_mu.p;
    za.sig = (const double *)pl->d_zl_sig.p;
    za.slice = (const int *)pl->d_zl_slice.p;
    za.J = (const int *)pl->d_zl_J.p;
    za.tab0 = (const int *)pl->d_zl_tab0.p;
    za.sig0 = (const int *)pl->d_zl_sig0.p;
    za.npad = npad;
    za.mp0 = mp0;
    za.mstride = L.mstride;
    za.ncmax = L.ncmax;
    za.m0 = (int)L.m[0];
    za.m1 = (int)L.m[1];
    const bool t = pl->ev_used * 2 + 1 < (int64_t)pl->ev.size();
    FPS_HIP(fps::launch_zeig_lds(za, (int)npad, st, t ? pl->ev[2 * pl->ev_used] : nullptr,
                                 t ? pl->ev[2 * pl->ev_used + 1] : nullptr));
    if (t) ++pl->ev_used;
  } else {
    // Per-slice ADI, all active slices per launch.
    const int K = (int)pl->zslice.size();
    const int nsw = pl->zsw_start[0], nrd = pl->zrd_start[0];
    const fps::BatchSweep *dsw = (const fps::BatchSweep *)pl->d_zsw.p;
    const fps::BatchReduce *drd = (const fps::BatchReduce *)pl->d_zrd.p;
    const int *swmap = (const int *)pl->d_zswmap.p, *rdmap = (const int *)pl->d_zrdmap.p;
    fps::SweepArgs plain{}, stencil{};
    stencil.pre = (const double *)pl->d_pre.p;
    // sweep launch, timed with the plan's event pairs while they last
    // (rows: the x solves, row-chain batches)
    auto sweep = [&](const fps::SweepArgs &types, bool with_g, const fps::BatchSweep *d, int nwg,
                     int wg_base, hipStream_t s2, bool rows = false) -> hipError_t {
      const bool t = pl->ev_used * 2 + 1 < (int64_t)pl->ev.size();
      hipEvent_t e0 = t ? pl->ev[2 * pl->ev_used] : nullptr;
      hipEvent_t e1 = t ? pl->ev[2 * pl->ev_used + 1] : nullptr;
      const hipError_t e =
          rows ? fps::launch_sweep_batch_rows(types, d, swmap, nwg, w, s2, wg_base, e0, e1)
               : fps::launch_sweep_batch(types, with_g, d, swmap, nwg, w, s2, wg_base, e0, e1);
      if (t && e == hipSuccess) ++pl->ev_used;
      return e;
    };
    // All steps of sorted slices lo .. hi-1 on stream s2: at step j the
    // active ones are lo .. min(zactive[j], hi) - 1 (J descending).
    auto run_group = [&](int lo, int hi, hipStream_t s2) -> hipError_t {
      hipError_t e = hipSuccess;
      for (int j = 0; j < pl->zJmax && e == hipSuccess; ++j) {
        const int k1 = std::min(pl->zactive[j], hi);
        if (k1 <= lo) break;
        const size_t o1 = ((size_t)j * 2 + 0) * K, o2 = ((size_t)j * 2 + 1) * K;
        e = sweep(plain, false, dsw + o1, (k1 - lo) * nsw, lo * nsw, s2, true);
        if (e == hipSuccess && !pl->zfused)
          e = fps::launch_reduce_batch(drd + o1, rdmap, (k1 - lo) * nrd, L.ncmax, w, s2, lo * nrd);
        // y solves: stencil P = A~ + mu before the solve, the identity for
        // the slices at their last step, all in one launch
        if (e == hipSuccess) e = sweep(stencil, true, dsw + o2, (k1 - lo) * nsw, lo * nsw, s2);
        if (e == hipSuccess && !pl->zfused)
          e = fps::launch_reduce_batch(drd + o2, rdmap, (k1 - lo) * nrd, L.ncmax, w, s2, lo * nrd);
      }
      return e;
    };
    // The longest slices iterate on the plan's side stream beside the rest, so
    // their short launches at the end overlap the bulk; launches timed per
    // dispatch all go to the caller's stream.
    if (pl->zsplit > 0 && pl->zsplit < K && pl->zside && pl->ev.empty()) {
      // One solve at a time forks onto the side stream, so the event
      // records and waits of concurrent host threads do not interleave.  The
      // join is enqueued whatever the groups returned, so the side stream
      // (or a graph being captured) is never left forked.
      std::lock_guard<std::mutex> lk(pl->zlock);
      FPS_HIP(hipEventRecord(pl->zfork, st));
      FPS_HIP(hipStreamWaitEvent(pl->zside, pl->zfork, 0));
      const hipError_t e1 = run_group(0, pl->zsplit, pl->zside);
      const hipError_t e2 = e1 == hipSuccess ? run_group(pl->zsplit, K, st) : hipSuccess;
      const hipError_t e3 = hipEventRecord(pl->zjoin, pl->zside);
      const hipError_t e4 = e3 == hipSuccess ? hipStreamWaitEvent(st, pl->zjoin, 0) : e3;
      FPS_HIP(e1);
      FPS_HIP(e2);
      FPS_HIP(e3);
      FPS_HIP(e4);
    } else {
      FPS_HIP(run_group(0, K, st));
    }
    if (pl->zfused)  // the carries of every slice's last half-step, in one launch
      FPS_HIP(fps::launch_reduce_batch((const fps::BatchReduce *)pl->d_zrdfin.p, rdmap, K * nrd,
                                       L.ncmax, w, st));
    FPS_HIP(fps::launch_slice_final<double>(O1, (const double *)(w + pl->off_ab),
                                            (const double *const *)pl->d_zfin.p, Yh, -1.0, 0, npad,
                                            mp0, L.mstride, L.ncmax, st));
  }
  // Output.
  if (pl->out_basis == FPS_OUT_NATIVE) {
    const double *MV[2] = {(const double *)pl->d_Vz[0].p, (const double *)pl->d_Vz[1].p};
    std::vector<fps::GemmProb> pz;
    mode_probs(Yh, full, O0, full, 0, MV, ldm, MV, ldm, Nfull, K2, pz);
    if ((s = launch_probs(pz, st)) != FPS_OK) return s;
    FPS_HIP(fps::launch_permute3_out(O0, U, L.n, npad, mp0, (const double *)pl->d_sinv.p, st));
    return FPS_OK;
  }
  const int64_t mq = pl->mqc[0] + pl->mqc[1], mb0 = pl->mqc[0];
  const double *MB[2] = {(const double *)pl->d_PB[0].p, (const double *)pl->d_PB[1].p};
  const double *MPV[2] = {(const double *)pl->d_PV[0].p, (const double *)pl->d_PV[1].p};
  const int64_t ldb[2] = {pl->mop[0], pl->mop[1]};
  const int64_t N[2] = {L.m[0] > 0 ? L.mo[0] : 0, L.m[1] > 0 ? L.mo[1] : 0};
  const Dims d1{{npad, npad, mq}, {mp0, mp0, mb0}};
  const Dims d2{{npad, mq, mq}, {mp0, mb0, mb0}};
  const Dims d3{{mq, mq, mq}, {mb0, mb0, mb0}};
  std::vector<fps::GemmProb> px, pz;
  const bool empty_block = L.m[0] == 0 || L.m[1] == 0;  // n = 1: see cube_solve
  if (empty_block) FPS_HIP(fps::launch_fill(O0, npad * npad * mq, 0.0, st));
  mode_probs(Yh, full, O0, d1, 2, MB, ldm, MB, ldb, N, K2, px);
  if ((s = launch_probs(px, st)) != FPS_OK) return s;
  if (empty_block) FPS_HIP(fps::launch_fill(RX, npad * mq * mq, 0.0, st));
  FPS_HIP(fps::launch_gemm_table((const fps::GemmDesc *)pl->d_gy_out.p,
                                 (const int *)pl->d_gy_map_out.p, pl->gy_tiles[1], w, nullptr, st));
  if (empty_block) FPS_HIP(fps::launch_fill(O0, mq * mq * mq, 0.0, st));
  mode_probs(RX, d2, O0, d3, 0, MPV, ldm, MPV, ldb, N, K2, pz);
  if ((s = launch_probs(pz, st)) != FPS_OK) return s;
  FPS_HIP(fps::launch_permute3_out(O0, U, L.n + 2, mq, mb0, nullptr, st));
  return FPS_OK;
}

}  // namespace detail
}  // namespace fps
