// Internal interfaces shared by the C ABI translation units (not part of
// the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fps.h"
#include "kernels.hpp"
#include "planner.hpp"

namespace fps {
namespace detail {

// Records `msg` as the calling thread's last error and returns `s`.
fps_status fail(fps_status s, const std::string &msg);
const char *last_error();

#define FPS_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::fps::detail::fail(FPS_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr uint64_t kMagic = 0x66707370'6c616e31ull;  // "fpsplan1"

struct DeviceBuf {
  void *p = nullptr;
  DeviceBuf() = default;
  DeviceBuf(const DeviceBuf &) = delete;
  DeviceBuf &operator=(const DeviceBuf &) = delete;
  ~DeviceBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace detail
}  // namespace fps

struct CylPlan;  // cylinder plans (cylinder.cpp)

struct fps_plan {
  uint64_t magic = fps::detail::kMagic;
  CylPlan *cyl = nullptr;  // non-null for cylinder plans
  fps_plan() = default;
  fps_plan(const fps_plan &) = delete;
  fps_plan &operator=(const fps_plan &) = delete;
  ~fps_plan();
  int dim = 2;
  int64_t n = 0;
  double tol = 0;
  int prec = FPS_FP64;
  int out_basis = FPS_OUT_CHEB;
  unsigned flags = 0;
  bool on_device = false;

  fps::ShiftSet shifts;     // shifts of the ADI the sweeps run (FP32_REFINED: of round 0)
  // Refinement rounds (FP32_REFINED; FP64 plans have one round, the plain
  // ADI): round k runs an ADI to rtol[k] with the shifts rsh[k], whose step j
  // uses the tables of step rbase[k] + j; with rf32[k] set it stores every
  // sweep array in float.  n_f32 counts the steps of the float rounds.
  int rounds = 1;
  std::vector<fps::ShiftSet> rsh;
  std::vector<int> rbase;
  std::vector<double> rtol;
  std::vector<char> rf32;
  int n_f32 = 0;

  // Rectangle [a, b] x [c, d] (rect plans): the symmetric form reads
  // sx2 A~ Y + sy2 Y A~ = G with sx2 = (2/(b-a))^2, sy2 = (2/(d-c))^2, i.e.
  // A Y - Y B = G for A = sx2 A~ (rows), B = -sy2 A~ (columns).  ADI step j
  // then solves with two matrices: table 2j holds sy2 A~ + p_j (first
  // half-step), table 2j + 1 holds sx2 A~ - q_j (second half-step).  The
  // square uses one table per step (A~ + p_j, q_j = -p_j) and sx2 = sy2 = 1.
  bool rect = false;
  double box[4] = {-1.0, 1.0, -1.0, 1.0};
  double sx2 = 1.0, sy2 = 1.0;
  int tab1(int j) const { return rect ? 2 * j : j; }
  int tab2(int j) const { return rect ? 2 * j + 1 : j; }
  fps::Layout L;
  std::vector<double> tab, ctab, l1;  // host sweep tables
  std::vector<double> sdiag, soff;          // A~ stencil in the parity-blocked layout
  std::vector<double> Rs[2], P[2];  // host conversion maps (unpadded)
  int64_t mop[2] = {0, 0};          // output parity lengths padded to 64
  std::vector<double> sinv;         // 1/sqrt((i+1)(i+2))

  // device copies
  fps::detail::DeviceBuf d_tab, d_ctab, d_l1, d_sinv, d_sdiag, d_soff;
  // GEMM operands, zero-padded to multiples of 64: RsA = Rs (mp x mp),
  // RsB = Rs^T (mp x mp), PA = P (mop x mp), PB = P^T (mp x mop).
  fps::detail::DeviceBuf d_RsA[2], d_RsB[2], d_PA[2], d_PB[2];
  // Lift map S^-1 C~(T_k'') by parity (m[s] x mo[s], row-major), only with
  // FPS_PLAN_DIRICHLET.
  fps::detail::DeviceBuf d_lift[2];

  // sweep timing diagnostics
  std::vector<hipEvent_t> ev;  // pairs
  int64_t ev_used = 0;

  // workspace layout (byte offsets)
  int64_t off_G = 0, off_GT = 0, off_O0 = 0, off_O1 = 0, off_lv = 0, off_ab = 0;
  // Second chunk-boundary-value buffer: 2-D plans' second half-steps write
  // lv2 and first ones lv; z-eigenbasis cube plans whose sweeps form their
  // carries themselves use it the same way.  2-D plans: the carries of first
  // half-steps go to ab2, those of second ones (and the final pass's) to ab,
  // so that the two row-parity halves of the ADI can run on two streams
  // without sharing a buffer element.
  int64_t off_lv2 = 0, off_ab2 = 0;
  int64_t off_X = 0;  // adjoint: the output cotangent in the parity-blocked layout
  int64_t off_R = 0;  // FP32_REFINED: the float residual and its transpose
  // Dirichlet lift (2-D plans with FPS_PLAN_DIRICHLET): the traces' scaled
  // C~ second-derivative coefficients [4][npad] (parity-blocked) and their
  // values at -1 and +1 [8].
  int64_t off_bc = 0;

  // Cube (dim 3), two-level nested ADI: `shifts` holds the outer shifts
  // (p in [-2/delta, -2], q in [1, 1/delta]); inner step (i, j) has shift
  // inner_p[inner_off[i] + j]; sweep table id of the z pass of outer step i
  // is i, of inner step (i, j) it is J + inner_off[i] + j.
  std::vector<int> inner_J, inner_off;
  std::vector<double> inner_p;
  double cube_inner_tol = 0.0;
  int64_t mqc[2] = {0, 0};  // compact output parity sizes (mo rounded up to even)
  fps::detail::DeviceBuf d_pre;             // [2][npad]: A~ diagonal and coupling per row
  fps::detail::DeviceBuf d_RbA[2], d_RbB[2];  // input map A~^-1 S^-1 R blocks and transposes
  fps::detail::DeviceBuf d_gy_in, d_gy_out;   // mode-y GEMM tables (input / output map)
  int gy_tiles[2] = {0, 0};
  fps::detail::DeviceBuf d_gy_map_in, d_gy_map_out;
  int64_t off_ZR = 0, off_RX = 0, off_RXT = 0;

  // Cube, z-eigenbasis method (FPS_PLAN_CUBE_ZEIG): slice k of the sorted
  // active slices (J descending) is storage slice zslice[k], eigenvalue
  // zmu[k], zJ[k] ADI steps with table ids ztab0[k] + 2 j (x solve) and
  // ztab0[k] + 2 j + 1 (y solve).
  bool zeig = false;
  std::vector<int> zslice, zJ, ztab0, zactive, zsw_start, zrd_start;
  // Sweeps form their own chunk carries (chains of at most two chunks,
  // ncmax <= 2): no carry launch between half-steps, one per solve (FP64) or
  // per round (refined) before the final pass, from the descriptors d_zrdfin.
  bool zfused = false;
  fps::detail::DeviceBuf d_zrdfin;
  std::vector<double> zmu;
  std::vector<double> zp, zq;  // shifts of step j of sorted slice k at index ztab0[k] / 2 + j
  int zJmax = 0;
  fps::detail::DeviceBuf d_zsw, d_zrd, d_zswmap, d_zrdmap, d_zfin;
  // FP64 plans whose parity blocks fit one workgroup's LDS (n <= 256): the
  // whole slice ADI as one launch of k_zeig_lds, over the sorted slices and
  // then the inactive storage slices (zl_slice, zl_J, zl_tab0, zl_sig0 per
  // entry; zl_mu the shifts mu; zl_sig the two sigmas of every step).
  bool zlds = false;
  // Nested cube plans whose parity blocks fit one workgroup's LDS: every
  // outer step's inner ADI is one k_zeig_lds launch (d_zl_tab32 / ctab32 the
  // chunk multipliers of every table, d_zl_sig the inner sigmas, outer step i
  // at 2 inner_off[i]).
  bool nlds = false;
  fps::detail::DeviceBuf d_zl_slice, d_zl_J, d_zl_tab0, d_zl_sig0, d_zl_mu, d_zl_sig;
  fps::detail::DeviceBuf d_zl_tab32, d_zl_ctab32;  // the kernel's chunk multipliers
  // Sorted slices 0 .. zsplit-1 (the longest) iterate on the plan's own
  // stream zside, the others on the caller's stream, joined by the events
  // zfork / zjoin (zsplit 0: one stream).
  int zsplit = 0;
  hipStream_t zside = nullptr;
  hipEvent_t zfork = nullptr, zjoin = nullptr;
  // Held while one solve enqueues its fork, both slice groups and its join,
  // so concurrent host threads' solves do not interleave on zside.
  std::mutex zlock;
  fps::detail::DeviceBuf d_Mz[2], d_PV[2], d_Vz[2];  // z maps: V^T S^-1 R, P V, V
  // Refined z-eigenbasis plans (FPS_FP32_REFINED): round r corrects Y^ by
  // solving, on every slice, (|mu| K + 1/2) dY + dY (|mu| K + 1/2) = K q K
  // (K = -A~^-1, q the negated slice residual) with its own shifts; sorted
  // slice k (|mu| descending) is storage slice zrslice[k] with zrJ[r][k]
  // steps on tables zrtab0[r][k] + j; step j of round r has descriptor row
  // zrrow0[r] + j and zractive[r][j] slices still iterating.  Table 0 is A~
  // itself (the two solves that form K q K).
  std::vector<int> zrslice;
  std::vector<double> zrmu_slice;  // mu of every storage slice (0 for padding)
  std::vector<std::vector<int>> zrJ, zrtab0, zractive;
  std::vector<int> zrJmax, zrrow0;
  // per round: sorted slices 0 .. zrsplit[r]-1 iterate on the side stream
  // (zside / zfork / zjoin, as zsplit for FP64 plans); 0: one stream
  std::vector<int> zrsplit;
  fps::detail::DeviceBuf d_zrsw, d_zrrd, d_zrfin, d_zmu;
  std::vector<double> zV[2];  // host eigenvectors of the parity blocks (m x m, columns)
  int64_t ws_bytes = 0;

  const double *tab_dev(int j) const {
    return (const double *)d_tab.p + (size_t)j * 2 * fps::kNTab * L.mstride;
  }
  const double *ctab_dev(int j) const {
    return (const double *)d_ctab.p + (size_t)j * 2 * fps::kNCTab * L.ncmax;
  }
  const double *l1_dev(int j) const {
    return (const double *)d_l1.p + (size_t)j * 2 * L.ncmax * fps::kL1;
  }
};

namespace fps {
namespace detail {

bool valid_plan(const fps_plan *p);
// Enclosure [a, b] of sigma(A~) (both negative) from the computed extreme
// eigenvalues, widened by a relative 1e-6.
void spectrum_tight(int64_t n, double *a, double *b);
int64_t align256(int64_t x);
template <typename T>
fps_status upload(DeviceBuf &b, const std::vector<T> &h) {
  if (h.empty()) return FPS_OK;
  if (hipMalloc(&b.p, h.size() * sizeof(T)) != hipSuccess)
    return fail(FPS_E_NOMEM, "hipMalloc of a plan table failed");
  FPS_HIP(hipMemcpy(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return FPS_OK;
}
// The refinement rounds of an FP32_REFINED plan with target tolerance tol:
// each round's inner ADI tolerance and whether it stores its sweep arrays in
// float (Dirichlet plans end with an FP64 round).
struct RefineRound {
  double tol;
  bool f32;
};
std::vector<RefineRound> refine_schedule(double tol, bool dirichlet);
// Input map of one square or rectangle problem: F (n x n, natural order) ->
// G and G^T in the plan's workspace `ws`; with `bc` non-null, G also takes
// the Dirichlet lift's correction (the traces' values at -1 and +1 are kept
// in the workspace for the output correction).
fps_status rhs_transform(fps_plan *pl, const double *F, char *ws, hipStream_t st,
                         const double *bc = nullptr);
// The coefficient-map GEMMs of one problem (up to 4 parity-block products
// per stage; returns their count), operands formed from the workspace base
// `ws` (and Y, U); rhs: g1 then g2 after k_permute_in of F into the GT
// region; out: g1 then g2 after U is zero-filled.
int rhs_gemms(const fps_plan *pl, char *ws, fps::GemmProb *g1, fps::GemmProb *g2);
int out_gemms(const fps_plan *pl, const double *Y, double *U, char *ws, fps::GemmProb *g1,
              fps::GemmProb *g2);
// Output map: Y (parity-blocked) -> U in the plan's output basis.
fps_status out_transform(fps_plan *pl, const double *Y, double *U, char *ws, hipStream_t st);
// Y of A~ Y + Y A~ = G for G in the workspace (FP64 or refined).
fps_status solve_symmetric(fps_plan *pl, char *w, hipStream_t st, double **Yout);
// The adjoint's maps around the ADI (transposes of the input and output
// maps): adjoint_in forms Ybar from Ubar into the G region (and G^T);
// adjoint_out forms Fbar from the ADI output Gbar.  FP64 plans.
fps_status adjoint_in(const fps_plan *pl, const double *Ubar, char *w, hipStream_t st);
// Pieces of the two for the batched adjoint: the input map up to its GEMMs
// (permutation, clear of G; native: the whole map), and the GEMMs of the
// input map (Chebyshev output only) and of the output map, built like
// rhs_gemms / out_gemms.
fps_status adjoint_in_pre(const fps_plan *pl, const double *Ubar, char *w, hipStream_t st);
int adj_in_gemms(const fps_plan *pl, char *w, fps::GemmProb *g1, fps::GemmProb *g2);
int adj_out_gemms(const fps_plan *pl, const double *Yb, double *Fbar, char *w, fps::GemmProb *g1,
                  fps::GemmProb *g2);
fps_status adjoint_out(const fps_plan *pl, const double *Gbar, double *Fbar, char *w,
                       hipStream_t st);
// Cube: host tables and workspace layout (after the common fields are set),
// their upload, and the solve.
fps_status cube_plan_build(fps_plan *pl);
fps_status cube_plan_upload(fps_plan *pl);
fps_status cube_solve(fps_plan *pl, const double *F, double *U, char *ws, hipStream_t st);
hipError_t timed_sweep(fps_plan *pl, const fps::SweepArgs &a, hipStream_t st, bool rows = false);
// The plan's default-priority side stream and its fork / join events
// (zside / zfork / zjoin), created once.
fps_status create_side_stream(fps_plan *pl);
// Cylinder (Sec. 4.1): host tables and workspace layout, their upload, the
// solve, and the band of one mode's r-operators (inspection).
fps_status cyl_plan_build(fps_plan *pl, int64_t nt);
fps_status cyl_plan_upload(fps_plan *pl);
fps_status cyl_solve(fps_plan *pl, const double *F, double *U, char *ws, hipStream_t st);
int64_t cyl_ws_bytes(const fps_plan *pl);
int64_t cyl_out_entries(const fps_plan *pl);
void cyl_mode_bands(int64_t n, int64_t kabs, std::vector<double> &Pb, std::vector<double> &Qb);

}  // namespace detail
}  // namespace fps
