// Test-only C shim over the host planner (built with g++ by the CPU tests).
#include <cstring>
#include <vector>

#include "../paper_1710_11259_amd/csrc/launch_limits.hpp"
#include "../paper_1710_11259_amd/csrc/planner.hpp"

extern "C" {
int shim_elem_launch_fits(long long workgroups) { return fps::elem_launch_fits(workgroups) ? 1 : 0; }
void shim_layout(long long n, long long *out) {
  fps::Layout L = fps::make_layout(n);
  long long v[] = {L.m[0], L.m[1], L.mp[0], L.mp[1], L.npad, L.nc[0], L.nc[1], L.ncmax,
                   L.mstride, L.mo[0], L.mo[1], fps::kSeg, fps::kWaves, fps::kChunk};
  std::memcpy(out, v, sizeof(v));
}
void shim_tables(long long n, int J, const double *p, double *pos, double *chunk) {
  fps::Layout L = fps::make_layout(n);
  std::vector<double> pv(p, p + J), a, b, cmb, l1;
  fps::build_sweep_tables(L, pv, a, b, cmb, l1);
  std::memcpy(pos, a.data(), a.size() * sizeof(double));
  std::memcpy(chunk, b.data(), b.size() * sizeof(double));
}
// The chunk multipliers of `chunk`-position chunks (the LDS-resident slice
// kernel's) for the sweep tables of shifts p.
void shim_chunk_tables(long long n, int J, const double *p, long long chunk, double *pos,
                       double *ch) {
  fps::Layout L = fps::make_layout(n);
  std::vector<double> pv(p, p + J), a, b, cmb, l1, tp, tc;
  fps::build_sweep_tables(L, pv, a, b, cmb, l1);
  fps::build_chunk_tables(L, a, chunk, tp, tc);
  std::memcpy(pos, tp.data(), tp.size() * sizeof(double));
  std::memcpy(ch, tc.data(), tc.size() * sizeof(double));
}
void shim_comb(long long n, int J, const double *p, double *comb) {
  fps::Layout L = fps::make_layout(n);
  std::vector<double> pv(p, p + J), a, b, cmb, l1;
  fps::build_sweep_tables(L, pv, a, b, cmb, l1);
  std::memcpy(comb, cmb.data(), cmb.size() * sizeof(double));
}
void shim_conversions(long long n, double *R0, double *R1, double *P0, double *P1) {
  fps::Layout L = fps::make_layout(n);
  std::vector<double> Rs[2], P[2];
  fps::build_conversions(L, Rs, P);
  std::memcpy(R0, Rs[0].data(), Rs[0].size() * sizeof(double));
  std::memcpy(R1, Rs[1].data(), Rs[1].size() * sizeof(double));
  std::memcpy(P0, P[0].data(), P[0].size() * sizeof(double));
  std::memcpy(P1, P[1].data(), P[1].size() * sizeof(double));
}
void shim_lift_map(long long n, double *M0, double *M1) {
  fps::Layout L = fps::make_layout(n);
  std::vector<double> Ms[2];
  fps::build_lift_map(L, Ms);
  std::memcpy(M0, Ms[0].data(), Ms[0].size() * sizeof(double));
  std::memcpy(M1, Ms[1].data(), Ms[1].size() * sizeof(double));
}
// Eigen-decomposition of the parity-s block of A~: m eigenvalues, m x m vectors.
int shim_atilde_eigen(long long n, int s, double *lam, double *Q) {
  const long long m = (n - s + 1) / 2;
  std::vector<long double> d(m), e(m > 1 ? m - 1 : 0), q;
  for (long long k = 0; k < m; ++k) d[k] = fps::atilde_diag(2 * k + s);
  for (long long k = 0; k + 1 < m; ++k) e[k] = fps::atilde_off(2 * k + s);
  if (!fps::tridiag_eigen(d, e, q)) return 0;
  for (long long k = 0; k < m; ++k) lam[k] = (double)d[k];
  for (long long k = 0; k < m * m; ++k) Q[k] = (double)q[k];
  return 1;
}

void shim_extremes(long long n, double *out) {
  long double lo, hi;
  fps::atilde_extremes(n, &lo, &hi);
  out[0] = (double)lo;
  out[1] = (double)hi;
}

int shim_dn(double alpha, int J, double *dn) {
  long double m1 = 1.0L / ((long double)alpha * alpha);
  long double K = fps::ellip_K_comp(m1);
  for (int j = 0; j < J; ++j) dn[j] = (double)fps::ellip_dn_comp((j + 0.5L) * K / J, m1, K);
  return 0;
}
}
