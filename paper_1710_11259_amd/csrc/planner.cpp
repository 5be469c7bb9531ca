// Host planner: shifts, iteration count, sweep tables, coefficient maps.
#include "planner.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace fps {

namespace {

// Carlson's symmetric integral R_F(x, y, z) by the duplication theorem
// (B. C. Carlson, Numer. Algorithms 10 (1995)), in extended precision.
long double carlson_rf(long double x, long double y, long double z) {
  for (int it = 0; it < 200; ++it) {
    const long double sx = std::sqrt(x), sy = std::sqrt(y), sz = std::sqrt(z);
    const long double lam = sx * sy + sy * sz + sz * sx;
    x = 0.25L * (x + lam);
    y = 0.25L * (y + lam);
    z = 0.25L * (z + lam);
    const long double A = (x + y + z) / 3.0L;
    const long double X = 1.0L - x / A, Y = 1.0L - y / A, Z = -X - Y;
    const long double dev = std::max(std::fabs(X), std::max(std::fabs(Y), std::fabs(Z)));
    if (dev < 1e-4L) {
      const long double E2 = X * Y - Z * Z, E3 = X * Y * Z;
      return (1.0L - E2 / 10.0L + E3 / 14.0L + E2 * E2 / 24.0L - 3.0L * E2 * E3 / 44.0L) /
             std::sqrt(A);
    }
  }
  return std::numeric_limits<long double>::quiet_NaN();
}

// dn(u | m), m = 1 - m1, for 0 <= u <= K/2.  The amplitude is written as
// phi = pi/2 - t; t solves F(pi/2 - t | m) = u with
// F = cos t R_F(sin^2 t, sin^2 t + m1 cos^2 t, 1) and dF/dt = -1/dn, by
// Newton's method from the m = 1 limit t = 2 atan(exp(-u)).  Then
// dn = sqrt(sin^2 t + m1 cos^2 t); no quantity is formed as 1 - m.
long double dn_newton(long double u, long double m1) {
  long double t = 2.0L * std::atan(std::exp(-u));
  for (int it = 0; it < 60; ++it) {
    const long double st = std::sin(t), ct = std::cos(t);
    const long double d2 = st * st + m1 * ct * ct;
    const long double F = ct * carlson_rf(st * st, d2, 1.0L);
    const long double step = (F - u) * std::sqrt(d2);
    t += step;
    if (std::fabs(step) <= 4 * std::numeric_limits<long double>::epsilon() * (t + 1e-30L)) break;
  }
  const long double st = std::sin(t), ct = std::cos(t);
  return std::sqrt(st * st + m1 * ct * ct);
}
}  // namespace

double cross_ratio(double a, double b, double c, double d) {
  return std::fabs(c - a) * std::fabs(d - b) / (std::fabs(c - b) * std::fabs(d - a));
}

int iteration_count(double a, double b, double c, double d, double tol) {
  if (!(tol > 0.0 && tol < 1.0)) return -1;
  if (!(a < b && b < c && c < d)) return -1;
  if (!std::isfinite(a) || !std::isfinite(d)) return -1;
  const double g = cross_ratio(a, b, c, d);
  const double pi = 3.141592653589793;
  double x = std::log(16.0 * g) * std::log(4.0 / tol) / (pi * pi);
  if (!std::isfinite(x) || x > 1e7) return -1;
  int J = (int)std::ceil(x);
  return J < 1 ? 1 : J;
}

long double ellip_K_comp(long double m1) { return carlson_rf(0.0L, m1, 1.0L); }

long double ellip_dn_comp(long double u, long double m1, long double K) {
  // dn(u) dn(K - u) = k' = sqrt(m1): evaluate on the half [0, K/2] only.
  if (u > 0.5L * K) return std::sqrt(m1) / dn_newton(K - u, m1);
  return dn_newton(u, m1);
}

bool zolotarev_shifts(double a, double b, double c, double d, double tol, ShiftSet &out,
                      std::string &err) {
  int J = iteration_count(a, b, c, d, tol);
  if (J < 0) {
    err = "invalid enclosure or tolerance: need a < b < c < d finite and 0 < tol < 1";
    return false;
  }
  const long double g = cross_ratio(a, b, c, d);
  const long double alpha = -1.0L + 2.0L * g + 2.0L * std::sqrt(g * g - g);
  const long double m1 = 1.0L / (alpha * alpha);
  // K and dn in the complementary parameter m1 = 1/alpha^2 for every alpha:
  // neither forms 1 - m1, so no separate large-alpha evaluation is needed
  // (m1 reaches ~1e-41 for the square enclosure at n = 2e5, far inside the
  // extended-precision range).
  std::vector<long double> dn(J);
  const long double K = ellip_K_comp(m1);
  for (int j = 0; j < J; ++j) dn[j] = ellip_dn_comp((j + 0.5L) * K / J, m1, K);
  out.J = J;
  out.p.resize(J);
  out.q.resize(J);
  if (c == -b && d == -a) {
    // Symmetric intervals: the Moebius map is odd, T(z) = c z and c alpha = d.
    for (int j = 0; j < J; ++j) {
      out.p[j] = (double)(-(long double)d * dn[j]);
      out.q[j] = -out.p[j];
    }
    return true;
  }
  // General case: T = W^-1 o Z, Z sends (-alpha, -1, 1) to (0, 1, inf),
  // W sends (a, b, c) to (0, 1, inf); both as 2x2 coefficient matrices.
  auto to_std = [](long double z1, long double z2, long double z3, long double Mx[4]) {
    Mx[0] = z2 - z3;
    Mx[1] = -z1 * (z2 - z3);
    Mx[2] = z2 - z1;
    Mx[3] = -z3 * (z2 - z1);
  };
  long double Zm[4], Wm[4];
  to_std(-alpha, -1.0L, 1.0L, Zm);
  to_std(a, b, c, Wm);
  long double Wi[4] = {Wm[3], -Wm[1], -Wm[2], Wm[0]};  // adjugate = inverse up to scale
  long double T[4] = {Wi[0] * Zm[0] + Wi[1] * Zm[2], Wi[0] * Zm[1] + Wi[1] * Zm[3],
                      Wi[2] * Zm[0] + Wi[3] * Zm[2], Wi[2] * Zm[1] + Wi[3] * Zm[3]};
  auto Tz = [&](long double z) { return (T[0] * z + T[1]) / (T[2] * z + T[3]); };
  for (int j = 0; j < J; ++j) {
    out.p[j] = (double)Tz(-alpha * dn[j]);
    out.q[j] = (double)Tz(alpha * dn[j]);
  }
  return true;
}

Layout make_layout(int64_t n) {
  Layout L;
  L.n = n;
  L.m[0] = (n + 1) / 2;
  L.m[1] = n / 2;
  for (int s = 0; s < 2; ++s) {
    L.mp[s] = (L.m[s] + kPad - 1) / kPad * kPad;
    L.nc[s] = (L.mp[s] + kChunk - 1) / kChunk;
    L.mo[s] = (n + 2 - s + 1) / 2;
  }
  L.npad = L.mp[0] + L.mp[1];
  L.ncmax = std::max(L.nc[0], L.nc[1]);
  L.mstride = L.ncmax * kChunk;
  return L;
}

double atilde_diag(int64_t i) {
  const double x = (double)i;
  return -2.0 / ((2 * x + 1) * (2 * x + 5));
}

double atilde_off(int64_t i) {
  const double x = (double)i;
  return 1.0 / ((2 * x + 5) * std::sqrt((2 * x + 3) * (2 * x + 7)));
}

namespace {

// Number of eigenvalues below x of the parity-s block of A~ (m positions):
// the negative pivots of the LDL^T factorization of the block minus x I.
int64_t sturm_count(int64_t m, int s, long double x) {
  int64_t cnt = 0;
  long double q = 1.0L;
  // a zero pivot counts as negative (x just above an eigenvalue): replaced by
  // a tiny negative value, 2^-13000 (about 1e-3913, far below any pivot but
  // with e^2 / q still finite in extended precision)
  const long double tiny = std::ldexp(1.0L, -13000);
  for (int64_t k = 0; k < m; ++k) {
    const long double d = (long double)atilde_diag(2 * k + s) - x;
    if (k == 0) {
      q = d;
    } else {
      const long double e = atilde_off(2 * (k - 1) + s);
      q = d - e * e / q;
    }
    if (q == 0.0L) q = -tiny;
    if (q < 0.0L) ++cnt;
  }
  return cnt;
}

}  // namespace

bool tridiag_eigen(std::vector<long double> &d, std::vector<long double> e,
                   std::vector<long double> &Q) {
  const int64_t m = (int64_t)d.size();
  Q.assign((size_t)(m * m), 0.0L);
  for (int64_t i = 0; i < m; ++i) Q[(size_t)(i * m + i)] = 1.0L;
  e.resize(m > 0 ? m : 1, 0.0L);
  const long double eps = std::numeric_limits<long double>::epsilon();
  auto negligible = [&](int64_t k) {  // coupling of k and k+1
    return std::fabs(e[k]) <= eps * (std::fabs(d[k]) + std::fabs(d[k + 1]));
  };
  int64_t h = m - 1, iters = 0;
  while (h > 0) {
    if (negligible(h - 1)) {
      e[h - 1] = 0.0L;
      --h;
      continue;
    }
    if (++iters > 60 * m) return false;
    int64_t l = h - 1;
    while (l > 0 && !negligible(l - 1)) --l;
    // Wilkinson shift: eigenvalue of the trailing 2 x 2 block nearer d[h].
    const long double t = 0.5L * (d[h - 1] - d[h]);
    const long double eh = e[h - 1];
    const long double den = t + (t >= 0 ? 1.0L : -1.0L) * std::sqrt(t * t + eh * eh);
    const long double mu = d[h] - eh * eh / den;
    // Bulge chase with Givens rotations G = [[c, s], [-s, c]] on (k, k+1):
    // new basis vectors c v_k - s v_{k+1} and s v_k + c v_{k+1}.
    long double x = d[l] - mu, z = e[l], bulge = 0.0L;
    for (int64_t k = l; k < h; ++k) {
      long double c, sn;
      if (k == l) {
        const long double r = std::sqrt(x * x + z * z);
        c = x / r;
        sn = -z / r;
      } else {
        const long double r = std::sqrt(e[k - 1] * e[k - 1] + bulge * bulge);
        c = e[k - 1] / r;
        sn = -bulge / r;
        e[k - 1] = r;
      }
      const long double a = d[k], b = e[k], cc = d[k + 1];
      d[k] = c * c * a - 2.0L * c * sn * b + sn * sn * cc;
      d[k + 1] = sn * sn * a + 2.0L * c * sn * b + c * c * cc;
      e[k] = c * sn * (a - cc) + (c * c - sn * sn) * b;
      if (k + 1 < h) {
        bulge = -sn * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      for (int64_t i = 0; i < m; ++i) {
        long double *row = &Q[(size_t)(i * m)];
        const long double qk = row[k], qk1 = row[k + 1];
        row[k] = c * qk - sn * qk1;
        row[k + 1] = sn * qk + c * qk1;
      }
    }
  }
  // ascending order
  std::vector<int64_t> idx(m);
  for (int64_t i = 0; i < m; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return d[a] < d[b]; });
  std::vector<long double> d2(m), Q2((size_t)(m * m));
  for (int64_t j = 0; j < m; ++j) {
    d2[j] = d[idx[j]];
    for (int64_t i = 0; i < m; ++i) Q2[(size_t)(i * m + j)] = Q[(size_t)(i * m + idx[j])];
  }
  d.swap(d2);
  Q.swap(Q2);
  return true;
}

void atilde_extremes(int64_t n, long double *lmin, long double *lmax) {
  // Lemma B.1 encloses the spectrum in [-1, 0); bisect each parity block's
  // extreme eigenvalues inside it.
  long double lo_all = 0.0L, hi_all = -1.0L;
  for (int s = 0; s < 2; ++s) {
    const int64_t m = (n - s + 1) / 2;
    if (m == 0) continue;
    long double lo = -1.0L, hi = 0.0L;  // smallest: count(x) >= 1
    for (int it = 0; it < 200; ++it) {
      const long double mid = 0.5L * (lo + hi);
      if (sturm_count(m, s, mid) >= 1) hi = mid; else lo = mid;
    }
    lo_all = std::min(lo_all, lo);
    lo = -1.0L, hi = 0.0L;  // largest: count(x) == m
    for (int it = 0; it < 200; ++it) {
      const long double mid = 0.5L * (lo + hi);
      if (sturm_count(m, s, mid) >= m) hi = mid; else lo = mid;
    }
    hi_all = std::max(hi_all, hi);
  }
  *lmin = lo_all;
  *lmax = hi_all;
}

void build_sweep_tables(const Layout &L, const std::vector<double> &p, std::vector<double> &pos,
                        std::vector<double> &chunk, std::vector<double> &comb,
                        std::vector<double> &l1) {
  build_sweep_tables_ab(L, std::vector<double>(p.size(), 1.0), p, pos, chunk, &comb, l1);
}

void build_chunk_tables(const Layout &L, const std::vector<double> &pos, int64_t chunk,
                        std::vector<double> &out_pos, std::vector<double> &out_chunk) {
  const int64_t ms = L.mstride, nq = ms / chunk;
  const size_t J = pos.size() / (size_t)(2 * kNTab * ms);
  out_pos.assign(J * 2 * 2 * (size_t)ms, 0.0);
  out_chunk.assign(J * 2 * 3 * (size_t)nq, 0.0);
  std::vector<long double> F2((size_t)ms);
  for (size_t j = 0; j < J; ++j)
    for (int s = 0; s < 2; ++s) {
      const double *T = pos.data() + (j * 2 + s) * kNTab * (size_t)ms;
      const double *l = T + T_L * ms, *ib = T + T_IB * ms, *u = T + T_U * ms;
      double *P = out_pos.data() + (j * 2 + s) * 2 * (size_t)ms;
      double *C = out_chunk.data() + (j * 2 + s) * 3 * (size_t)nq;
      for (int64_t c = 0; c < nq; ++c) {
        const int64_t c0 = c * chunk, c1 = c0 + chunk;
        long double acc = 1.0L;
        for (int64_t k = c0; k < c1; ++k) {
          acc *= -(long double)l[k];
          F2[(size_t)k] = acc;
        }
        long double x = 0.0L, bk = 1.0L;
        for (int64_t k = c1 - 1; k >= c0; --k) {
          x = F2[(size_t)k] * (long double)ib[k] - (long double)u[k] * x;
          bk *= -(long double)u[k];
          P[k] = (double)x;        // BF2
          P[ms + k] = (double)bk;  // Bk2
        }
        C[c] = (double)F2[(size_t)(c1 - 1)];  // F2last
        C[nq + c] = P[c0];                    // BF2first
        C[2 * nq + c] = P[ms + c0];           // Bk2first
      }
    }
}

void build_sweep_tables_ab(const Layout &L, const std::vector<double> &alpha,
                           const std::vector<double> &beta0, std::vector<double> &pos,
                           std::vector<double> &chunk, std::vector<double> *combp,
                           std::vector<double> &l1) {
  std::vector<double> unused;
  std::vector<double> &comb = combp ? *combp : unused;
  const int J = (int)alpha.size();
  const int64_t ms = L.mstride, nc = L.ncmax;
  pos.assign((size_t)J * 2 * kNTab * ms, 0.0);
  chunk.assign((size_t)J * 2 * kNCTab * nc, 0.0);
  if (combp) comb.assign((size_t)J * 2 * nc * nc * kNComb, 0.0);
  l1.assign((size_t)J * 2 * nc * kL1, 0.0);
  std::vector<long double> CF((size_t)(nc + 1) * nc), CBY((size_t)nc * nc), CBX((size_t)nc * nc);
  std::vector<long double> l(ms), ib(ms), u(ms), F2(ms), BF2(ms);
  for (int j = 0; j < J; ++j) {
    for (int s = 0; s < 2; ++s) {
      const int64_t m = L.m[s];
      double *T = pos.data() + ((size_t)(j * 2 + s) * kNTab) * ms;
      double *C = chunk.data() + ((size_t)(j * 2 + s) * kNCTab) * nc;
      std::fill(l.begin(), l.end(), 0.0L);
      std::fill(ib.begin(), ib.end(), 0.0L);
      std::fill(u.begin(), u.end(), 0.0L);
      if (m == 0) continue;
      // Thomas factors of (alpha_j A~ + beta_j I) restricted to parity s.
      const long double al = alpha[j], be = beta0[j];
      long double beta = al * (long double)atilde_diag(s) + be;
      ib[0] = 1.0L / beta;
      for (int64_t k = 1; k < m; ++k) {
        const long double e = al * (long double)atilde_off(2 * (k - 1) + s);
        l[k] = e * ib[k - 1];
        beta = (al * (long double)atilde_diag(2 * k + s) + be) - l[k] * e;
        ib[k] = 1.0L / beta;
      }
      for (int64_t k = 0; k + 1 < m; ++k)
        u[k] = al * (long double)atilde_off(2 * k + s) * ib[k];
      for (int64_t k = 0; k < ms; ++k) {
        T[T_L * ms + k] = (double)l[k];
        T[T_IB * ms + k] = (double)ib[k];
        T[T_U * ms + k] = (double)u[k];
      }
      // Segment multipliers.
      for (int64_t s0 = 0; s0 < ms; s0 += kSeg) {
        long double acc = 1.0L;
        for (int64_t k = s0; k < s0 + kSeg; ++k) {
          acc *= -l[k];
          T[T_F1 * ms + k] = (double)acc;
        }
        acc = 1.0L;
        for (int64_t k = s0 + kSeg - 1; k >= s0; --k) {
          acc *= -u[k];
          T[T_BK1 * ms + k] = (double)acc;
        }
      }
      // Chunk multipliers.
      for (int64_t c = 0; c < nc; ++c) {
        const int64_t c0 = c * kChunk, c1 = c0 + kChunk;
        long double acc = 1.0L;
        for (int64_t k = c0; k < c1; ++k) {
          acc *= -l[k];
          F2[k] = acc;
        }
        long double x = 0.0L;
        for (int64_t k = c1 - 1; k >= c0; --k) {
          x = F2[k] * ib[k] - u[k] * x;
          BF2[k] = x;
        }
        acc = 1.0L;
        for (int64_t k = c1 - 1; k >= c0; --k) {
          acc *= -u[k];
          T[T_BK2 * ms + k] = (double)acc;
          T[T_BF2 * ms + k] = (double)BF2[k];
        }
        C[C_F2LAST * nc + c] = (double)F2[c1 - 1];
        C[C_BF2FIRST * nc + c] = (double)BF2[c0];
        C[C_BK2FIRST * nc + c] = T[T_BK2 * ms + c0];
      }
      // Segment-carry combinations inside each chunk.
      for (int64_t cc = 0; cc < nc; ++cc) {
        double *Lc = l1.data() + ((size_t)(j * 2 + s) * nc + cc) * kL1;
        const int64_t c0 = cc * kChunk;
        for (int w = 0; w < kWaves; ++w)
          for (int u = 0; u < kWaves; ++u) {
            long double f = 0.0L, b = 0.0L;
            if (u < w) {
              f = 1.0L;
              for (int v = u + 1; v < w; ++v) f *= T[T_F1 * ms + c0 + (int64_t)v * kSeg + kSeg - 1];
            }
            if (u > w) {
              b = 1.0L;
              for (int v = w + 1; v < u; ++v) b *= T[T_BK1 * ms + c0 + (int64_t)v * kSeg];
            }
            Lc[(0 * kWaves + w) * kWaves + u] = (double)f;
            Lc[(1 * kWaves + w) * kWaves + u] = (double)b;
          }
      }
      if (!combp) continue;
      // Coefficients of the chunk carries as linear forms in the boundary
      // values: cf[0] = 0, cf[c+1] = ylast[c] + F2last[c] cf[c];
      // cb[ncs-1] = 0, cb[c] = xfirst[c+1] + BF2first[c+1] cf[c+1] + Bk2first[c+1] cb[c+1].
      const int64_t ncs = L.nc[s];
      std::fill(CF.begin(), CF.end(), 0.0L);
      std::fill(CBY.begin(), CBY.end(), 0.0L);
      std::fill(CBX.begin(), CBX.end(), 0.0L);
      for (int64_t cc = 0; cc + 1 < ncs; ++cc) {
        const long double f = C[C_F2LAST * nc + cc];
        for (int64_t q = 0; q < nc; ++q) CF[(cc + 1) * nc + q] = f * CF[cc * nc + q];
        CF[(cc + 1) * nc + cc] += 1.0L;
      }
      for (int64_t cc = ncs - 2; cc >= 0; --cc) {
        const long double bf = C[C_BF2FIRST * nc + cc + 1], bk = C[C_BK2FIRST * nc + cc + 1];
        for (int64_t q = 0; q < nc; ++q) {
          CBY[cc * nc + q] = bf * CF[(cc + 1) * nc + q] + bk * CBY[(cc + 1) * nc + q];
          CBX[cc * nc + q] = bk * CBX[(cc + 1) * nc + q];
        }
        CBX[cc * nc + cc + 1] += 1.0L;
      }
      double *W = comb.data() + (size_t)(j * 2 + s) * nc * nc * kNComb;
      for (int64_t cc = 0; cc < ncs; ++cc)
        for (int64_t q = 0; q < ncs; ++q) {
          W[(cc * nc + q) * kNComb + K_CF] = (double)CF[cc * nc + q];
          W[(cc * nc + q) * kNComb + K_CBY] = (double)CBY[cc * nc + q];
          W[(cc * nc + q) * kNComb + K_CBX] = (double)CBX[cc * nc + q];
        }
    }
  }
}

void build_conversions(const Layout &L, std::vector<double> Rs[2], std::vector<double> P[2]) {
  const int64_t n = L.n, N = n + 2;
  auto beta = [](int64_t i) -> long double {
    const long double x = (long double)i;
    return std::sqrt((x + 1) * (x + 3) / ((2 * x + 3) * (2 * x + 5)));
  };
  auto sc = [](int64_t i) -> long double {
    const long double x = (long double)i;
    return std::sqrt((x + 1) * (x + 2));
  };
  for (int s = 0; s < 2; ++s) {
    Rs[s].assign((size_t)L.m[s] * L.m[s], 0.0);
    P[s].assign((size_t)L.mo[s] * L.m[s], 0.0);
  }
  // Input map: C~ coefficients of T_k by T_{k+1} = 2 x T_k - T_{k-1}, with
  // multiplication by x in the C~ basis: x C~_i = beta_i C~_{i+1} + beta_{i-1} C~_{i-1}.
  {
    std::vector<long double> prev(n + 1, 0.0L), cur(n + 1, 0.0L), nxt(n + 1, 0.0L);
    auto emit = [&](int64_t k, const std::vector<long double> &v) {
      const int s = (int)(k & 1);
      const int64_t b = k >> 1, ms = L.m[s];
      for (int64_t i = s; i <= k; i += 2) Rs[s][(size_t)(i >> 1) * ms + b] = (double)(v[i] / sc(i));
    };
    auto jx = [&](const std::vector<long double> &v, int64_t deg, std::vector<long double> &w) {
      // w = x * v for v with nonzeros at indices <= deg (same parity as deg)
      for (int64_t i = 0; i <= deg + 1 && i <= n; ++i) w[i] = 0.0L;
      for (int64_t i = deg & 1; i <= deg; i += 2) {
        if (i + 1 <= n) w[i + 1] += beta(i) * v[i];
        if (i >= 1) w[i - 1] += beta(i - 1) * v[i];
      }
    };
    cur[0] = 2.0L / std::sqrt(3.0L);
    emit(0, cur);
    if (n > 1) {
      jx(cur, 0, nxt);
      std::swap(prev, cur);
      std::swap(cur, nxt);
      emit(1, cur);
    }
    for (int64_t k = 1; k + 1 < n; ++k) {
      jx(cur, k, nxt);
      for (int64_t i = (k + 1) & 1; i <= k + 1; i += 2) nxt[i] = 2.0L * nxt[i] - prev[i];
      std::swap(prev, cur);
      std::swap(cur, nxt);
      emit(k + 1, cur);
    }
  }
  // Output map: Chebyshev coefficients of phi_i = (1-x^2) C~_i by the same
  // three-term recurrence, phi_{i+1} = (x phi_i - beta_{i-1} phi_{i-1}) / beta_i,
  // with x T_0 = T_1 and x T_k = (T_{k+1} + T_{k-1}) / 2.
  {
    std::vector<long double> prev(N + 1, 0.0L), cur(N + 1, 0.0L), nxt(N + 1, 0.0L);
    auto emit = [&](int64_t i, const std::vector<long double> &v) {
      const int s = (int)(i & 1);
      const int64_t b = i >> 1, ms = L.m[s];
      for (int64_t k = s; k <= std::min(i + 2, N - 1); k += 2)
        P[s][(size_t)(k >> 1) * ms + b] = (double)(v[k] / sc(i));
    };
    auto xt = [&](const std::vector<long double> &v, int64_t deg, std::vector<long double> &w) {
      for (int64_t k = 0; k <= deg + 1 && k <= N; ++k) w[k] = 0.0L;
      for (int64_t k = deg & 1; k <= deg; k += 2) {
        if (k == 0) {
          w[1] += v[0];
        } else {
          if (k + 1 <= N) w[k + 1] += 0.5L * v[k];
          w[k - 1] += 0.5L * v[k];
        }
      }
    };
    const long double h = std::sqrt(3.0L) / 4.0L;
    cur[0] = h;
    cur[2] = -h;
    emit(0, cur);
    if (n > 1) {
      xt(cur, 2, nxt);
      for (int64_t k = 0; k <= 3; ++k) nxt[k] /= beta(0);
      std::swap(prev, cur);
      std::swap(cur, nxt);
      emit(1, cur);
    }
    for (int64_t i = 1; i + 1 < n; ++i) {
      xt(cur, i + 2, nxt);
      const long double bi = beta(i), bm = beta(i - 1);
      for (int64_t k = (i + 1) & 1; k <= i + 3; k += 2) nxt[k] = (nxt[k] - bm * prev[k]) / bi;
      std::swap(prev, cur);
      std::swap(cur, nxt);
      emit(i + 1, cur);
    }
  }
}

void build_lift_map(const Layout &L, std::vector<double> Ms[2]) {
  const int64_t n = L.n, N = n + 2;
  for (int s = 0; s < 2; ++s) Ms[s].assign((size_t)L.m[s] * L.mo[s], 0.0);
  // T''_k = 2k C^(2)_{k-2} (d/dx T_k = k C^(1)_{k-1}, d/dx C^(l)_j = 2l C^(l+1)_{j-1});
  // C^(lam)_j = sum_l c_{j,l} C^(mu)_{j-2l} with (DLMF 18.18.16)
  //   c_{j,l} = (lam-mu)_l (lam)_{j-l} (mu + j - 2l) / ((mu)_{j-l+1} l!),
  // lam = 2, mu = 3/2; C^(3/2)_i = C~_i / nu_i, nu_i = sqrt((i+3/2)/((i+1)(i+2))).
  const long double lam = 2.0L, mu = 1.5L;
  long double u0 = 1.0L / mu;  // (lam)_j / (mu)_{j+1} at j = 0
  for (int64_t k = 2; k < N; ++k) {
    const int64_t j = k - 2;
    if (j > 0) u0 *= (lam + (long double)(j - 1)) / (mu + (long double)j);
    const int s = (int)(k & 1);
    long double u = u0;
    for (int64_t l = 0; 2 * l <= j; ++l) {
      const int64_t i = j - 2 * l;
      if (i < n) {
        const long double x = (long double)i;
        const long double nu = std::sqrt((x + 1.5L) / ((x + 1.0L) * (x + 2.0L)));
        const long double sc = std::sqrt((x + 1.0L) * (x + 2.0L));
        Ms[s][(size_t)(i >> 1) * L.mo[s] + (k >> 1)] =
            (double)(2.0L * (long double)k * u * (mu + x) / (nu * sc));
      }
      u *= (lam - mu + (long double)l) / (long double)(l + 1) * (mu + (long double)(j - l)) /
           (lam + (long double)(j - l - 1));
    }
  }
}

}  // namespace fps
