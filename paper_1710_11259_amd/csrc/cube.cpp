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
  std::vector<int> m(tiles);
  for (size_t k = 0; k < tab.size(); ++k) {
    const int end = k + 1 < tab.size() ? tab[k + 1].tile_start : tiles;
    std::fill(m.begin() + tab[k].tile_start, m.begin() + end, (int)k);
  }
  fps_status s;
  if ((s = upload(d, tab)) != FPS_OK || (s = upload(map, m)) != FPS_OK) return s;
  return FPS_OK;
}

Dims full_dims(const fps::Layout &L) {
  return Dims{{L.npad, L.npad, L.npad}, {L.mp[0], L.mp[0], L.mp[0]}};
}

}  // namespace

fps_status cube_plan_build(fps_plan *pl) {
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
  return FPS_OK;
}

fps_status cube_solve(fps_plan *pl, const double *F, double *U, char *w, hipStream_t st) {
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
    FPS_HIP(fps::launch_cube_zfinal(O0, ab, pl->tab_dev(i), RX, RXT, npad, mp0, L.mstride, L.ncmax,
                                    st));
    // (x, y) half-step: inner ADI on every z-slice
    const int J2 = pl->inner_J[i];
    const double *p2 = pl->inner_p.data() + pl->inner_off[i];
    const int t0 = J1 + pl->inner_off[i];
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
      FPS_HIP(fps::launch_reduce(lv, pl->ctab_dev(t), ab, -a.sigma, npad, a.nc0, a.nc1, L.ncmax, st,
                                 (int)npad, S.lvb, S.abb));
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
      FPS_HIP(fps::launch_reduce(lv, pl->ctab_dev(t), ab, last ? 1.0 : -b.sigma, npad, b.nc0, b.nc1,
                                 L.ncmax, st, (int)npad, S.lvb, S.abb));
    }
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
  mode_probs(ZR, full, O0, d1, 2, MA, ldm, MB, ldb, N, K, px);
  if ((s = launch_probs(px, st)) != FPS_OK) return s;
  FPS_HIP(fps::launch_gemm_table((const fps::GemmDesc *)pl->d_gy_out.p,
                                 (const int *)pl->d_gy_map_out.p, pl->gy_tiles[1], w, nullptr, st));
  mode_probs(RX, d2, O0, d3, 0, MA, ldm, MB, ldb, N, K, pz);
  if ((s = launch_probs(pz, st)) != FPS_OK) return s;
  FPS_HIP(fps::launch_permute3_out(O0, U, L.n + 2, mq, mb0, nullptr, st));
  return FPS_OK;
}

}  // namespace detail
}  // namespace fps
