// Poisson on the cylinder (Sec. 4.1): DFS-doubled data in Chebyshev (r) x
// Fourier (theta) x Chebyshev (z) coefficients, one two-dimensional system
// per Fourier mode k,
//   P_k Y M + Q_k Y D = R_k      (Y: C~(r) x C~(z) coefficients of w_k),
// with P_k, Q_k the Galerkin matrices of the mode's r-operators (partial
// regularity u~_k = r^m (1-r^2)(1-z^2) w_k, m = min(|k|, 2); the three
// cases of Sec. 4.1), M = [(1 - z^2)] and D of (3.6) in z.
//
// Method.  The z-operators are the same for every mode: with D = -S^2 and
// Y = Ybar S^-1 the system reads P Ybar A~ + Q Ybar = -R S^-1, and in the
// eigenbasis A~ = V diag(lambda) V^T of each z-parity block (Yhat = Ybar V)
// every column j is an independent banded system in r,
//   (Q_k + lambda_j P_k) yhat_j = -(R S^-1 V)_j,
// pentadiagonal in the parity-restricted r index.  The plan factors every
// (|k|, lambda_j) matrix on the host (extended precision, partial pivoting)
// and the device applies the factors, one thread per (mode, real/imaginary
// part, column).  The z maps (eigen-transform folded with the Chebyshev ->
// C~ and output maps) run as two large MFMA GEMMs, the r maps as one table
// GEMM per direction.  (The paper solves each mode by ADI with near-normal
// shifts; the z-eigenbasis makes the per-mode problem exact and banded.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "solver.hpp"

struct CylPlan {
  int64_t n = 0, nt = 0, m = 0, mp = 0, npad = 0;
  int64_t mo = 0, mop = 0, mobar = 0;  // z output per parity (n/2 + 1), padded
  int64_t ro = 0;                      // r output rows per parity ((n + 4) / 2)
  int64_t nk = 0;                      // distinct |k|: 0 .. nt/2
  std::vector<int> slot_idx, slot_group, slot_kabs;  // internal slot -> mode
  fps::detail::DeviceBuf d_slot_idx;
  fps::detail::DeviceBuf d_groups;  // fps::CylSolveGroup per |k| present
  int ngroups = 0;
  fps::detail::DeviceBuf d_fac;               // [nk][8][mp][npad]
  fps::detail::DeviceBuf d_win[2], d_wout[2];  // z maps (mp x mp, mp x mop)
  fps::detail::DeviceBuf d_rin[4], d_rout[4];  // r maps per group (mp x mp, ro x mp)
  fps::detail::DeviceBuf d_routT[4];           // transposed r output maps (mp x ro)
  fps::detail::DeviceBuf d_tin, d_tin_map, d_tout, d_tout_map;
  int tiles_in = 0, tiles_out = 0;
  // output maps split into whole MFMA tiles and thin edges: leading extents
  // of the z output (columns per parity) and the r output (rows per parity),
  // the edge descriptors (d_tout_edge: fps::CylEdge per r output problem;
  // d_zedge: the two z output problems at full size)
  int64_t mo_main = 0, ro_main = 0;
  fps::detail::DeviceBuf d_tout_edge, d_zedge;
  int n_tout = 0;
  int64_t off_X0 = 0, off_X1 = 0, ws_bytes = 0;
  int64_t x0_elems = 0;
};

fps_plan::~fps_plan() { delete cyl; }

namespace fps {
namespace detail {

namespace {

// Groups of modes: 0 |k| >= 2 even, 1 |k| >= 3 odd, 2 |k| = 1, 3 k = 0.
int group_of(int64_t kabs) { return kabs >= 2 ? (int)(kabs & 1) : (kabs == 1 ? 2 : 3); }
// Parity of the right-hand side rows (rp), of w (wp), output r power m.
void group_par(int g, int *rp, int *wp, int *mpow) {
  *rp = g == 1 || g == 2 ? 1 : 0;
  *wp = g == 1 ? 1 : 0;
  *mpow = g <= 1 ? 2 : (g == 2 ? 1 : 0);
}

typedef long double ld;

// Multiplication by r^q in the C~ basis (exact entries of the infinite
// operator): J^q with J the Jacobi matrix x C~_i = b_i C~_{i+1} + b_{i-1} C~_{i-1}.
struct Mult {
  int64_t N;
  std::vector<ld> P[5];  // dense N x N, powers 0..4
  explicit Mult(int64_t n) : N(n + 8) {
    std::vector<ld> b(N);
    for (int64_t i = 0; i < N; ++i) {
      const ld x = (ld)i;
      b[i] = std::sqrt((x + 1) * (x + 3) / ((2 * x + 3) * (2 * x + 5)));
    }
    for (auto &p : P) p.assign((size_t)(N * N), 0.0L);
    for (int64_t i = 0; i < N; ++i) P[0][(size_t)(i * N + i)] = 1.0L;
    for (int q = 1; q <= 4; ++q)
      for (int64_t i = 0; i < N; ++i)
        for (int64_t l = std::max<int64_t>(0, i - q); l <= std::min(N - 1, i + q); ++l) {
          ld s = 0.0L;  // (J^{q-1} J)[i][l] = J^{q-1}[i][l-1] b_{l-1} + J^{q-1}[i][l+1] b_l
          if (l >= 1) s += P[q - 1][(size_t)(i * N + l - 1)] * b[l - 1];
          if (l + 1 < N) s += P[q - 1][(size_t)(i * N + l + 1)] * b[l];
          P[q][(size_t)(i * N + l)] = s;
        }
  }
  // [c0 + c1 r + ... + c4 r^4][i][l]
  ld poly(const ld c[5], int64_t i, int64_t l) const {
    if (i < 0 || l < 0 || i >= N || l >= N) return 0.0L;
    ld s = 0.0L;
    for (int q = 0; q <= 4; ++q)
      if (c[q] != 0.0L) s += c[q] * P[q][(size_t)(i * N + l)];
    return s;
  }
};

ld nu(int64_t j) {
  const ld x = (ld)j;
  return std::sqrt((x + 1.5L) / ((x + 1) * (x + 2)));
}
// C~_l coefficient of C~_j': C~_j' = 3 nu_j C^(5/2)_{j-1} (NIST 18.9.19) and
// C^(lam+1)_k = sum_l (lam + k - 2l)/lam C^(lam)_{k-2l} (DLMF 18.18.16 with a
// unit parameter gap).
ld D1(int64_t l, int64_t j) {
  if (l < 0 || j - l < 1 || ((j - l) & 1) == 0) return 0.0L;
  return 2.0L * nu(j) * ((ld)l + 1.5L) / nu(l);
}
// C~_l coefficient of C~_j'': C~_j'' = 15 nu_j C^(7/2)_{j-2} and the
// connection with parameter gap 2, c = (l'+1)(mu+k-l'+1)(mu+k-2l')/(mu(mu+1)).
ld D2(int64_t l, int64_t j) {
  if (l < 0 || j - l < 2 || ((j - l) & 1) == 1) return 0.0L;
  const ld lp = (ld)((j - 2 - l) / 2);
  return 4.0L * nu(j) * (lp + 1.0L) * ((ld)j + 0.5L - lp) * ((ld)l + 1.5L) / nu(l);
}

// Galerkin entry of a2 w'' + a1 w' + a0 w: sum_l [a2][i][l] D2[l][j] + ...
ld op_entry(const Mult &Mu, const ld a2[5], const ld a1[5], const ld a0[5], int64_t i, int64_t j) {
  ld s = Mu.poly(a0, i, j);
  for (int64_t l = std::max<int64_t>(0, i - 4); l <= i + 4; ++l) {
    const ld d2 = D2(l, j), d1 = D1(l, j);
    if (d2 != 0.0L) s += Mu.poly(a2, i, l) * d2;
    if (d1 != 0.0L) s += Mu.poly(a1, i, l) * d1;
  }
  return s;
}

// Coefficients of the mode operators (r^0 .. r^4).
void mode_coeffs(int g, int64_t kabs, ld a2[5], ld a1[5], ld a0[5], ld q[5]) {
  for (int t = 0; t < 5; ++t) a2[t] = a1[t] = a0[t] = q[t] = 0.0L;
  const ld k2 = (ld)kabs * (ld)kabs;
  if (g <= 1) {  // L1 - k^2 (1 - r^2); Q = r^2 - r^4
    a2[2] = 1, a2[4] = -1, a1[1] = 5, a1[3] = -9, a0[0] = 4 - k2, a0[2] = -16 + k2;
    q[2] = 1, q[4] = -1;
  } else if (g == 2) {  // L3; Q = r - r^3
    a2[1] = 1, a2[3] = -1, a1[0] = 3, a1[2] = -7, a0[1] = -8;
    q[1] = 1, q[3] = -1;
  } else {  // L4; Q = r^2 - r^4
    a2[2] = 1, a2[4] = -1, a1[1] = 1, a1[3] = -5, a0[2] = -4;
    q[2] = 1, q[4] = -1;
  }
}

}  // namespace

namespace {

// Band (offsets -2..2 in the parity-restricted index) of P_k and Q_k:
// Pb[a][c], Qb[a][c], entry (row 2a + rp, column 2(a + c - 2) + wp).
void mode_bands(const Mult &Mu, int64_t n, int64_t kabs, std::vector<ld> &Pb,
                std::vector<ld> &Qb) {
  const int g = group_of(kabs);
  int rp, wp, mpow;
  group_par(g, &rp, &wp, &mpow);
  ld a2[5], a1[5], a0[5], q[5];
  mode_coeffs(g, kabs, a2, a1, a0, q);
  const int64_t m = n / 2;
  Pb.assign((size_t)(m * 5), 0.0L);
  Qb.assign((size_t)(m * 5), 0.0L);
  for (int64_t a = 0; a < m; ++a)
    for (int c = 0; c < 5; ++c) {
      const int64_t b = a + c - 2;
      if (b < 0 || b >= m) continue;
      const int64_t i = 2 * a + rp, j = 2 * b + wp;
      Pb[(size_t)(a * 5 + c)] = op_entry(Mu, a2, a1, a0, i, j);
      Qb[(size_t)(a * 5 + c)] = Mu.poly(q, i, j);
    }
}

}  // namespace

void cyl_mode_bands(int64_t n, int64_t kabs, std::vector<double> &Pb, std::vector<double> &Qb) {
  const Mult Mu(n);
  std::vector<ld> P, Q;
  mode_bands(Mu, n, kabs, P, Q);
  Pb.assign(P.begin(), P.end());
  Qb.assign(Q.begin(), Q.end());
}

namespace {

// LU with partial pivoting of the band matrix A = Q + lambda P (offsets
// -2..2), in extended precision.  Per position a: pivot offset (0, 1, 2),
// the two multipliers, 1/u_aa and the four superdiagonal entries of U.
bool band_lu(const std::vector<ld> &Pb, const std::vector<ld> &Qb, ld lambda, int64_t m,
             double *f[8], int64_t stride) {
  // window ab[a][c] = entry (a, a + c - 2), c in [0, 7)
  std::vector<ld> ab((size_t)(m * 7), 0.0L);
  for (int64_t a = 0; a < m; ++a)
    for (int c = 0; c < 5; ++c) ab[(size_t)(a * 7 + c)] = Qb[(size_t)(a * 5 + c)] + lambda * Pb[(size_t)(a * 5 + c)];
  auto at = [&](int64_t r, int64_t col) -> ld & { return ab[(size_t)(r * 7 + (col - r + 2))]; };
  for (int64_t a = 0; a < m; ++a) {
    int64_t p = a;
    ld best = std::fabs(at(a, a));
    for (int64_t r = a + 1; r <= std::min(a + 2, m - 1); ++r)
      if (std::fabs(at(r, a)) > best) {
        best = std::fabs(at(r, a));
        p = r;
      }
    if (best == 0.0L) return false;
    if (p != a)
      for (int64_t col = a; col <= std::min(a + 4, m - 1); ++col) std::swap(at(a, col), at(p, col));
    const ld piv = at(a, a);
    ld lm[2] = {0.0L, 0.0L};
    for (int64_t r = a + 1; r <= std::min(a + 2, m - 1); ++r) {
      const ld l = at(r, a) / piv;
      lm[r - a - 1] = l;
      at(r, a) = 0.0L;
      for (int64_t col = a + 1; col <= std::min(a + 4, m - 1); ++col) at(r, col) -= l * at(a, col);
    }
    f[0][a * stride] = (double)(p - a);
    f[1][a * stride] = (double)lm[0];
    f[2][a * stride] = (double)lm[1];
    f[3][a * stride] = (double)(1.0L / piv);
    for (int t = 1; t <= 4; ++t) f[3 + t][a * stride] = a + t < m ? (double)at(a, a + t) : 0.0;
  }
  return true;
}

}  // namespace

fps_status cyl_plan_build(fps_plan *pl, int64_t nt) {
  const int64_t n = pl->n;
  if (n < 2 || (n & 1)) return fail(FPS_E_ARG, "cylinder plans need an even n >= 2");
  if (nt < 2 || (nt & 1)) return fail(FPS_E_ARG, "cylinder plans need an even number of Fourier modes");
  if (n > 512 || nt > 1024)
    return fail(FPS_E_UNSUPPORTED, "cylinder plans are limited to n <= 512, n_theta <= 1024");
  CylPlan *c = new (std::nothrow) CylPlan();
  if (!c) return fail(FPS_E_NOMEM, "plan allocation failed");
  pl->cyl = c;
  c->n = n;
  c->nt = nt;
  c->m = n / 2;
  c->mp = (c->m + fps::kPad - 1) / fps::kPad * fps::kPad;
  c->npad = 2 * c->mp;
  c->mo = c->m + 1;
  c->mop = (c->mo + fps::kPad - 1) / fps::kPad * fps::kPad;
  c->mobar = 2 * c->mop;
  c->ro = (n + 4) / 2;
  c->nk = nt / 2 + 1;
  // slots sorted by group
  for (int g = 0; g < 4; ++g)
    for (int64_t idx = 0; idx < nt; ++idx) {
      const int64_t k = idx - nt / 2, kabs = k < 0 ? -k : k;
      if (group_of(kabs) != g) continue;
      c->slot_idx.push_back((int)idx);
      c->slot_group.push_back(g);
      c->slot_kabs.push_back((int)kabs);
    }
  const int64_t X = nt * 2 * c->npad * c->npad;
  c->x0_elems = std::max<int64_t>(X, nt * 2 * c->npad * c->mobar);
  c->off_X0 = 0;
  c->off_X1 = align256(c->x0_elems * 8);
  c->ws_bytes = c->off_X1 + align256(X * 8);
  return FPS_OK;
}

fps_status cyl_plan_upload(fps_plan *pl) {
  CylPlan *c = pl->cyl;
  const int64_t n = c->n, m = c->m, mp = c->mp, npad = c->npad;
  fps::Layout L = fps::make_layout(n);
  if (L.m[0] != m || L.m[1] != m || L.mp[0] != mp)
    return fail(FPS_E_STATE, "internal: cylinder layout");
  std::vector<double> Rs[2], P[2];
  fps::build_conversions(L, Rs, P);
  auto sc = [](int64_t i) { return std::sqrt((double)(i + 1) * (double)(i + 2)); };
  // z eigenbasis per parity
  std::vector<long double> lam[2], V[2];
  for (int s = 0; s < 2; ++s) {
    std::vector<long double> d(m), e(m > 1 ? m - 1 : 0);
    for (int64_t k = 0; k < m; ++k) d[k] = fps::atilde_diag(2 * k + s);
    for (int64_t k = 0; k + 1 < m; ++k) e[k] = fps::atilde_off(2 * k + s);
    if (!fps::tridiag_eigen(d, e, V[s])) return fail(FPS_E_STATE, "eigen-decomposition of A~ failed");
    lam[s] = d;
  }
  fps_status st;
  // z maps: W_in = -Rs^T V (mp x mp, B operand), W_out = V^T P^T (mp x mop)
  for (int s = 0; s < 2; ++s) {
    std::vector<double> win((size_t)(mp * mp), 0.0), wout((size_t)(mp * c->mop), 0.0);
    for (int64_t b = 0; b < m; ++b)      // Chebyshev z index (row of W_in)
      for (int64_t j = 0; j < m; ++j) {  // eigen index
        long double acc = 0.0L;
        for (int64_t a = 0; a < m; ++a) acc += (long double)Rs[s][(size_t)(a * m + b)] * V[s][(size_t)(a * m + j)];
        win[(size_t)(b * mp + j)] = (double)(-acc);
      }
    for (int64_t j = 0; j < m; ++j)
      for (int64_t o = 0; o < c->mo; ++o) {
        long double acc = 0.0L;
        for (int64_t a = 0; a < m; ++a) acc += V[s][(size_t)(a * m + j)] * (long double)P[s][(size_t)(o * m + a)];
        wout[(size_t)(j * c->mop + o)] = (double)acc;
      }
    if ((st = upload(c->d_win[s], win)) != FPS_OK || (st = upload(c->d_wout[s], wout)) != FPS_OK) return st;
  }
  // r maps per group
  const Mult Mu(n);
  for (int g = 0; g < 4; ++g) {
    int rp, wp, mpow;
    group_par(g, &rp, &wp, &mpow);
    // R block of parity rp (C~ coefficient 2a+rp of T_{2b+rp}), unscaled
    std::vector<long double> R((size_t)(m * m));
    for (int64_t a = 0; a < m; ++a)
      for (int64_t b = 0; b < m; ++b)
        R[(size_t)(a * m + b)] = (long double)Rs[rp][(size_t)(a * m + b)] * sc(2 * a + rp);
    std::vector<double> rin((size_t)(mp * mp), 0.0);
    for (int64_t a = 0; a < m; ++a)
      for (int64_t b = 0; b < m; ++b) {
        long double v = R[(size_t)(a * m + b)];
        if (g == 3) {  // [r^2] R
          const ld r2[5] = {0, 0, 1, 0, 0};
          v = 0.0L;
          for (int64_t a2 = std::max<int64_t>(0, a - 1); a2 <= std::min(m - 1, a + 1); ++a2)
            v += Mu.poly(r2, 2 * a, 2 * a2) * R[(size_t)(a2 * m + b)];
        }
        rin[(size_t)(a * mp + b)] = (double)v;
      }
    // output: Chebyshev coefficients of r^mpow (1 - r^2) C~_{2b+wp}; P[wp]
    // holds those of (1 - r^2) C~_i / sc(i) at Chebyshev index 2o + wp
    const int outp = (mpow + wp) & 1;
    std::vector<double> rout((size_t)(c->ro * mp), 0.0);
    for (int64_t b = 0; b < m; ++b) {
      std::vector<long double> t((size_t)(n + 5), 0.0L);
      for (int64_t o = 0; o < c->mo; ++o) t[(size_t)(2 * o + wp)] = (long double)P[wp][(size_t)(o * m + b)] * sc(2 * b + wp);
      for (int q = 0; q < mpow; ++q) {  // multiply by x: x T_0 = T_1, x T_k = (T_{k+1} + T_{k-1})/2
        std::vector<long double> u((size_t)(n + 5), 0.0L);
        for (int64_t k = 0; k + 1 < n + 5; ++k) {
          if (t[k] == 0.0L) continue;
          if (k == 0) {
            u[1] += t[0];
          } else {
            u[k + 1] += 0.5L * t[k];
            u[k - 1] += 0.5L * t[k];
          }
        }
        t.swap(u);
      }
      for (int64_t o = 0; o < c->ro; ++o) rout[(size_t)(o * mp + b)] = (double)t[(size_t)(2 * o + outp)];
    }
    std::vector<double> routT((size_t)(mp * c->ro), 0.0);
    for (int64_t o = 0; o < c->ro; ++o)
      for (int64_t b = 0; b < mp; ++b) routT[(size_t)(b * c->ro + o)] = rout[(size_t)(o * mp + b)];
    if ((st = upload(c->d_rin[g], rin)) != FPS_OK || (st = upload(c->d_rout[g], rout)) != FPS_OK ||
        (st = upload(c->d_routT[g], routT)) != FPS_OK)
      return st;
  }
  // banded LU factors per (|k|, z column)
  {
    std::vector<double> fac((size_t)(c->nk * 8 * mp * npad), 0.0);
    for (int64_t kabs = 0; kabs < c->nk; ++kabs) {
      std::vector<ld> Pb, Qb;
      mode_bands(Mu, n, kabs, Pb, Qb);
      for (int s = 0; s < 2; ++s)
        for (int64_t j = 0; j < m; ++j) {
          const int64_t zpos = s * mp + j;
          double *f[8];
          for (int t = 0; t < 8; ++t) f[t] = fac.data() + ((kabs * 8 + t) * mp) * npad + zpos;
          if (!band_lu(Pb, Qb, lam[s][(size_t)j], m, f, npad))
            return fail(FPS_E_STATE, "internal: singular cylinder mode matrix");
        }
    }
    if ((st = upload(c->d_fac, fac)) != FPS_OK) return st;
  }
  // slot table, and the solve groups: the (slot, part) rows sharing one |k|
  std::vector<fps::CylSolveGroup> groups;
  {
    std::vector<int> gid(c->nk, -1);
    for (size_t sl = 0; sl < c->slot_idx.size(); ++sl) {
      const int kabs = c->slot_kabs[sl];
      if (gid[kabs] < 0) {
        fps::CylSolveGroup e;
        for (int r = 0; r < fps::kCylRhs; ++r) e.sp[r] = -1;
        int rp, wp, mpow;
        group_par(c->slot_group[sl], &rp, &wp, &mpow);
        e.kabs = kabs;
        e.rp = rp;
        e.wp = wp;
        gid[kabs] = (int)groups.size();
        groups.push_back(e);
      }
      fps::CylSolveGroup &e = groups[gid[kabs]];
      for (int part = 0; part < 2; ++part) {
        int r = 0;
        while (r < fps::kCylRhs && e.sp[r] >= 0) ++r;
        if (r == fps::kCylRhs) return fail(FPS_E_STATE, "internal: cylinder solve group overflow");
        e.sp[r] = (int)sl * 2 + part;
      }
    }
  }
  c->ngroups = (int)groups.size();
  if ((st = upload(c->d_slot_idx, c->slot_idx)) != FPS_OK || (st = upload(c->d_groups, groups)) != FPS_OK)
    return st;
  // r-map GEMM tables (workspace / output offsets)
  const int64_t nt = c->nt, N2 = (n + 4) * (n + 2);
  std::vector<fps::GemmDesc> tin, tout;
  int tiles = 0;
  for (size_t sl = 0; sl < c->slot_idx.size(); ++sl) {
    const int g = c->slot_group[sl];
    int rp, wp, mpow;
    group_par(g, &rp, &wp, &mpow);
    const int outp = (mpow + wp) & 1;
    for (int part = 0; part < 2; ++part) {
      const int64_t blk = ((int64_t)sl * 2 + part) * npad;
      // RHS rows (rp block) = R_g X1[rp block]: A absolute, B / C in ws (X1 -> X0)
      fps::GemmProb q{(const double *)c->d_rin[g].p,
                      (const double *)(intptr_t)(c->off_X1 + (blk + rp * mp) * npad * 8),
                      (double *)(intptr_t)(c->off_X0 + (blk + rp * mp) * npad * 8), mp, npad, mp,
                      mp, 1, npad, 1, npad, 1, 0, 0, 0, 0, 0, 0, 0, 0};
      if (!fps::gemm_operands_ok(q)) return fail(FPS_E_STATE, "internal: cylinder GEMM operands");
      fps::GemmDesc e{q, 0, 1, 1, tiles, 0};
      tiles += fps::gemm_tiles(q, &e.ntx);
      tin.push_back(e);
    }
  }
  c->tiles_in = tiles;
  tiles = 0;
  for (size_t sl = 0; sl < c->slot_idx.size(); ++sl) {
    const int g = c->slot_group[sl];
    int rp, wp, mpow;
    group_par(g, &rp, &wp, &mpow);
    const int outp = (mpow + wp) & 1;
    const int64_t idx = c->slot_idx[sl];
    for (int part = 0; part < 2; ++part)
      for (int s = 0; s < 2; ++s) {
        const int64_t blk = ((int64_t)sl * 2 + part) * npad;
        // U rows of parity outp, z columns of parity s: Pr_g X0[wp block, z block s]
        fps::GemmProb q{(const double *)c->d_rout[g].p,
                        (const double *)(intptr_t)(c->off_X0 + ((blk + wp * mp) * c->mobar + s * c->mop) * 8),
                        (double *)(intptr_t)((((idx * 2 + part) * N2) + outp * (n + 2) + s) * 8), c->ro,
                        c->mo, mp, mp, 1, c->mobar, 1, 2 * (n + 2), 2, 0, 0, 0, 0, 0, 0, 0, 0};
        if (!fps::gemm_operands_ok(q)) return fail(FPS_E_STATE, "internal: cylinder GEMM operands");
        fps::GemmDesc e{q, 0, 1, 2, tiles, 0};
        tiles += fps::gemm_tiles(q, &e.ntx);
        tout.push_back(e);
      }
  }
  c->tiles_out = tiles;
  // main table: whole tiles only; the edge kernel reads the full problems
  c->mo_main = fps::gemm_main_extent(c->mo);
  c->ro_main = fps::gemm_main_extent(c->ro);
  c->n_tout = (int)tout.size();
  std::vector<fps::GemmDesc> tout_main = tout;
  tiles = 0;
  for (fps::GemmDesc &e : tout_main) {
    e.p.M = c->ro_main;
    e.p.N = c->mo_main;
    e.tile_start = tiles;
    tiles += fps::gemm_tiles(e.p, &e.ntx);
  }
  c->tiles_out = tiles;
  if (c->mo_main != c->mo || c->ro_main != c->ro) {
    // one edge descriptor per r output problem, in the same order as tout
    std::vector<fps::CylEdge> edges;
    for (size_t sl = 0; sl < c->slot_idx.size(); ++sl)
      for (int part = 0; part < 2; ++part)
        for (int s = 0; s < 2; ++s) {
          const fps::GemmDesc &e = tout[edges.size()];
          edges.push_back(fps::CylEdge{(const double *)c->d_rout[c->slot_group[sl]].p,
                                       (const double *)c->d_routT[c->slot_group[sl]].p,
                                       (int64_t)(intptr_t)e.p.B, (int64_t)(intptr_t)e.p.C / 8});
        }
    if ((st = upload(c->d_tout_edge, edges)) != FPS_OK) return st;
  }
  {
    // z output problems (workspace offsets: X1 -> X0) for the edge columns
    std::vector<fps::GemmDesc> z;
    const int64_t rows = c->nt * 2 * npad;
    for (int s = 0; s < 2; ++s) {
      const fps::GemmProb q{(const double *)(intptr_t)(c->off_X1 + s * mp * 8),
                            (const double *)c->d_wout[s].p,
                            (double *)(intptr_t)(c->off_X0 + s * c->mop * 8), rows, c->mo, mp, npad, 1,
                            c->mop, 1, c->mobar, 1, 0, 0, 0, 0, 0, 0, 0, 0};
      z.push_back(fps::GemmDesc{q, 1, 0, 1, 0, 0});
    }
    if (c->mo_main != c->mo && (st = upload(c->d_zedge, z)) != FPS_OK) return st;
  }
  if ((st = upload(c->d_tin, tin)) != FPS_OK ||
      (st = upload(c->d_tin_map, fps::gemm_table_map(tin))) != FPS_OK ||
      (st = upload(c->d_tout, tout_main)) != FPS_OK ||
      (st = upload(c->d_tout_map, fps::gemm_table_map(tout_main))) != FPS_OK)
    return st;
  (void)nt;
  return FPS_OK;
}

int64_t cyl_ws_bytes(const fps_plan *pl) { return pl->cyl->ws_bytes; }
int64_t cyl_out_entries(const fps_plan *pl) {
  return pl->cyl->nt * 2 * (pl->cyl->n + 4) * (pl->cyl->n + 2);
}

fps_status cyl_solve(fps_plan *pl, const double *F, double *U, char *w, hipStream_t st) {
  CylPlan *c = pl->cyl;
  const int64_t n = c->n, nt = c->nt, mp = c->mp, npad = c->npad;
  double *X0 = (double *)(w + c->off_X0), *X1 = (double *)(w + c->off_X1);
  const int64_t rows = nt * 2 * npad;
  // 1. F -> X0 [slot][part][r][z], parity-blocked, zero padded
  FPS_HIP(fps::launch_cyl_permute_in(F, X0, (const int *)c->d_slot_idx.p, n, nt, mp, st));
  // 2. z map: X1 = X0 W_in (per z parity block)
  {
    fps::GemmProb q[2];
    for (int s = 0; s < 2; ++s)
      q[s] = fps::GemmProb{X0 + s * mp, (const double *)c->d_win[s].p, X1 + s * mp, rows, mp, mp,
                           npad, 1, mp, 1, npad, 1, 0, 0, 0, 0, 0, 0, 0, 0};
    FPS_HIP(fps::launch_gemm(q, 2, st));
  }
  // 3. r map: X0[rp block] = R_g X1[rp block]
  FPS_HIP(fps::launch_gemm_table((const fps::GemmDesc *)c->d_tin.p, (const int *)c->d_tin_map.p,
                                 c->tiles_in, w, nullptr, st));
  // 4. banded solves: X1[wp block] = yhat
  FPS_HIP(fps::launch_cyl_solve(X0, X1, (const double *)c->d_fac.p,
                                (const fps::CylSolveGroup *)c->d_groups.p, c->ngroups, c->m, mp, st));
  // 5. z output map: X0 [slot][part][r][zout] = X1 W_out
  {
    fps::GemmProb q[2];
    for (int s = 0; s < 2; ++s)
      q[s] = fps::GemmProb{X1 + s * mp, (const double *)c->d_wout[s].p, X0 + s * c->mop, rows,
                           c->mo_main, mp, npad, 1, c->mop, 1, c->mobar, 1, 0, 0, 0, 0, 0, 0, 0, 0};
    FPS_HIP(fps::launch_gemm(q, 2, st));
    if (c->mo_main != c->mo)  // the last z column of every row: one wavefront per row
      FPS_HIP(fps::launch_gemm_edge_cols((const fps::GemmDesc *)c->d_zedge.p, 2, c->mo_main,
                                         (int)std::min<int64_t>(2048, (rows + 15) / 16), w, nullptr,
                                         st));
  }
  // 6. r output map into U (rows of the other parity stay zero)
  FPS_HIP(fps::launch_fill(U, nt * 2 * (n + 4) * (n + 2), 0.0, st));
  FPS_HIP(fps::launch_gemm_table((const fps::GemmDesc *)c->d_tout.p, (const int *)c->d_tout_map.p,
                                 c->tiles_out, w, (char *)U, st));
  if (c->mo_main != c->mo || c->ro_main != c->ro)
    FPS_HIP(fps::launch_cyl_redge((const fps::CylEdge *)c->d_tout_edge.p, c->n_tout, w, U, mp, c->ro,
                                  c->ro_main, c->mo, c->mo_main, c->mobar, 2 * (n + 2), st));
  return FPS_OK;
}

}  // namespace detail
}  // namespace fps
