// Host planner of the spectral Poisson solver: ADI iteration count and
// Zolotarev shifts (Theorem 2.1, (2.4), (2.9), App. A), the per-shift Thomas
// factor tables of the partitioned tridiagonal sweeps, and the dense
// coefficient maps Chebyshev -> C~^(3/2) (input) and recombined C~ ->
// Chebyshev (output).  Pure C++ (no HIP); float64 results, extended
// precision where recurrences accumulate.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fps {

// Sweep partition.  A chain of one parity is cut into lane segments of
// kSeg positions; kWaves consecutive segments form a chunk handled by one
// workgroup; chunks are joined through a second-level carry recurrence.
constexpr int kSeg = 8;
constexpr int kWaves = 8;
constexpr int kChunk = kSeg * kWaves;
constexpr int kCols = 64;   // chains per wavefront (one per lane)
constexpr int kPad = 64;    // parity blocks are padded to a multiple of this

// Per-position table slots (see build_sweep_tables).
enum TabSlot { T_L = 0, T_IB = 1, T_U = 2, T_F1 = 3, T_BK1 = 4, T_BF2 = 5, T_BK2 = 6, kNTab = 7 };
// Per-chunk table slots.
enum ChunkSlot { C_F2LAST = 0, C_BF2FIRST = 1, C_BK2FIRST = 2, kNCTab = 3 };
// Carry-combination slots: the chunk-level forward carry cf[c] and backward
// carry cb[c] of a chain are linear in its chunk boundary values ylast[q]
// (forward-eliminated value at the end of chunk q, zero chunk carries) and
// xfirst[q] (back-substituted value at the start of chunk q):
//   cf[c] = sum_q W[c][q][K_CF] ylast[q],
//   cb[c] = sum_q W[c][q][K_CBY] ylast[q] + W[c][q][K_CBX] xfirst[q].
enum CombSlot { K_CF = 0, K_CBY = 1, K_CBX = 2, kNComb = 3 };
// Segment-carry combinations inside a chunk (waves w, u < kWaves):
//   cf1[w] = sum_{u<w} L1[c][0][w][u] ylast_seg[u]    (forward carry into segment w)
//   cb1[w] = sum_{u>w} L1[c][1][w][u] xfirst_seg[u]   (backward carry into segment w)
// with L1[.][0][w][u] = prod_{u<v<w} F1(last position of segment v) and
//      L1[.][1][w][u] = prod_{w<v<u} Bk1(first position of segment v).
constexpr int kL1 = 2 * kWaves * kWaves;

struct ShiftSet {
  int J = 0;
  std::vector<double> p, q;
};

// gamma of Theorem 2.1 (cross-ratio of a, b, c, d).
double cross_ratio(double a, double b, double c, double d);

// (2.9): J = ceil(log(16 gamma) log(4/tol) / pi^2).  Returns -1 on bad input.
int iteration_count(double a, double b, double c, double d, double tol);

// Complete elliptic integral K(m) = R_F(0, m1, 1) and dn(u | m) for the
// parameter m = 1 - m1, given the complementary parameter m1 (never forms 1 - m1).
long double ellip_K_comp(long double m1);
long double ellip_dn_comp(long double u, long double m1, long double K);

// Shifts of Theorem 2.1 for sigma(A) in [a,b], sigma(B) in [c,d].
// Returns false (and sets err) on invalid input.
bool zolotarev_shifts(double a, double b, double c, double d, double tol, ShiftSet &out,
                      std::string &err);

// Layout of the parity-blocked internal arrays of a size-n square solve.
struct Layout {
  int64_t n = 0;
  int64_t m[2] = {0, 0};    // chain lengths: ceil(n/2), floor(n/2)
  int64_t mp[2] = {0, 0};   // padded to kPad
  int64_t npad = 0;         // mp[0] + mp[1]
  int64_t nc[2] = {0, 0};   // chunks per parity
  int64_t ncmax = 0;
  int64_t mstride = 0;      // table length per (shift, parity, slot)
  int64_t mo[2] = {0, 0};   // output rows per parity for the (n+2)-long Chebyshev index
};
Layout make_layout(int64_t n);

// Eigen-decomposition of a symmetric tridiagonal matrix (diagonal d[0..m-1],
// off-diagonal e[0..m-2]) by implicit QR steps with Wilkinson shifts and
// Givens rotations in extended precision.  On return d holds the
// eigenvalues in ascending order and Q (m x m, row-major) the orthonormal
// eigenvectors as columns.  Returns false if the iteration does not settle.
bool tridiag_eigen(std::vector<long double> &d, std::vector<long double> e,
                   std::vector<long double> &Q);

// Smallest and largest eigenvalue of A~ (n x n, both parity blocks) by
// Sturm-sequence bisection in extended precision; both are negative.
void atilde_extremes(int64_t n, long double *lmin, long double *lmax);

// Entries of A~ = -S^-1 M S^-1 (symmetric, zero +-1 diagonals):
// diagonal at index i, and coupling between i and i+2.
double atilde_diag(int64_t i);
double atilde_off(int64_t i);

// Tables for the shifted solves (A~ + p I) along chains of one parity.
// pos:   [J][2][kNTab][mstride]; chunk: [J][2][kNCTab][ncmax];
// comb:  [J][2][ncmax][ncmax][kNComb];
// l1:    [J][2][ncmax][kL1].
// For chain position k (original index 2k + s), b_k = d_k + p, e_k the
// coupling to k+1.  Thomas over the whole chain: l_k = e_{k-1}/beta_{k-1},
// beta_k = b_k - l_k e_{k-1}, ib_k = 1/beta_k, u_k = e_k/beta_k.  Partition
// multipliers: F1_k = prod_{segment start..k} (-l), Bk1_k = prod_{k..segment
// end} (-u), BF2 = chunk-local backward solve of F2_k = prod_{chunk
// start..k} (-l) with zero carry at the chunk end, Bk2_k = prod_{k..chunk
// end} (-u).  Padded positions hold l = ib = u = 0 (inert).
void build_sweep_tables(const Layout &L, const std::vector<double> &p, std::vector<double> &pos,
                        std::vector<double> &chunk, std::vector<double> &comb,
                        std::vector<double> &l1);
// The same tables for the matrices alpha_j A~ + beta_j I (one per entry of
// alpha and beta); build_sweep_tables is the case alpha_j = 1, beta_j = p_j.
// comb may be null: the chunk-carry linear forms are then not built (the
// device evaluates the chunk-level recurrences from the chunk tables).
void build_sweep_tables_ab(const Layout &L, const std::vector<double> &alpha,
                           const std::vector<double> &beta, std::vector<double> &pos,
                           std::vector<double> &chunk, std::vector<double> *comb,
                           std::vector<double> &l1);

// Chunk multipliers of the tables `pos` ([J][2][kNTab][mstride], as built
// above) for chunks of `chunk` positions (a divisor of kChunk): per table
// and parity, BF2 and Bk2 at every position (out_pos [J][2][2][mstride]) and
// F2last, BF2first, Bk2first of every chunk (out_chunk [J][2][3][nq], nq =
// mstride / chunk), formed in extended precision from the stored l, ib, u.
void build_chunk_tables(const Layout &L, const std::vector<double> &pos, int64_t chunk,
                        std::vector<double> &out_pos, std::vector<double> &out_chunk);

// Conversion maps split by parity (row-major, float64):
//   Rs[s]: m[s] x m[s], Rs[s][a][b] = R[2a+s][2b+s] / sqrt((2a+s+1)(2a+s+2)),
//          R[i][k] = C~_i coefficient of T_k (upper triangular).
//   P[s]:  mo[s] x m[s], P[s][a][b] = Chebyshev coefficient 2a+s of
//          (1-x^2) C~_{2b+s}(x) / sqrt((2b+s+1)(2b+s+2)).
void build_conversions(const Layout &L, std::vector<double> Rs[2], std::vector<double> P[2]);

// Dirichlet lift map (Sec. 6.1): the scaled C~ coefficients of the second
// derivative of each Chebyshev polynomial, split by parity (row-major,
// float64, m[s] x mo[s]):
//   Ms[s][a][b] = C~_{2a+s} coefficient of T''_{2b+s} / sqrt((2a+s+1)(2a+s+2)),
// nonzero only for b > a.  From T''_k = 2k C^(2)_{k-2} and the Gegenbauer
// connection C^(2) -> C^(3/2) (all coefficients positive), accumulated in
// extended precision.  Applying it to a trace g gives S^-1 C~(g'') without
// forming g'' (whose C~ projection cancels heavily for rough g).
void build_lift_map(const Layout &L, std::vector<double> Ms[2]);

}  // namespace fps
