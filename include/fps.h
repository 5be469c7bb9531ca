/*
 * fps.h -- C ABI of the MI355X spectral fast Poisson solver.
 *
 * Method: Fortunato & Townsend, "Fast Poisson solvers for spectral methods"
 * (arXiv 1710.11259).  Poisson's equation u_xx + u_yy (+ u_zz) = f on
 * [-1,1]^dim with zero Dirichlet data (Sec. 3, (3.1); Sec. 5, (5.1)) is
 * discretized in the recombined basis (1-x^2) C~_j^(3/2)(x) of (3.2), giving
 * the generalized Sylvester equation (3.6) M X D^T + D X M^T = F.  After the
 * symmetrization of (3.9) (read as a congruence, X = S^-1 Y S^-1 with
 * S = |D|^(1/2)) the equation A~ Y + Y A~ = G is solved by the ADI iteration
 * of Algorithm 2 with the Zolotarev shifts of Theorem 2.1 (2.4) and the
 * iteration count (2.9), on the spectral enclosure [-1, -1/(30 n^4)] of
 * Lemma B.1.  Each shifted solve is a pair of tridiagonal (Thomas) solves,
 * one per parity (property P3, Sec. 3.3; App. B decoupling).
 *
 * Conventions
 *   - All arrays are float64, C-contiguous (row-major).
 *   - dim = 2: F[j*n + k] is the coefficient of T_j(y) T_k(x) (rows <-> y,
 *     as in (3.2)).  U has (n+2) x (n+2) entries, the exact Chebyshev
 *     coefficients of u (u has degree n+1 in each variable); with
 *     FPS_OUT_NATIVE, U has n x n entries, the coefficients X of (3.2).
 *   - dim = 3: F[(i*n + j)*n + k] multiplies T_i(z) T_j(y) T_k(x); U is
 *     (n+2)^3 (or n^3 native).
 *   - "dev" pointers are device memory on the current HIP device; "host"
 *     pointers are host memory.  `stream` is a hipStream_t (NULL = default).
 *   - Ownership: the caller owns F, U, the workspace and the stream.  A plan
 *     owns its host tables and the device copies of its constant tables; they
 *     are released by fps_plan_destroy.  Solves allocate no memory.
 *   - Errors: every call returns a status; nothing aborts.  Argument errors
 *     are reported synchronously.  Kernel faults surface as FPS_E_HIP from a
 *     later call or from the caller's synchronization.  fps_last_error()
 *     returns a thread-local message for the last failing call.
 *   - Concurrency: plans are immutable after creation; concurrent solves on
 *     one plan need distinct workspaces.
 */
#ifndef FPS_H
#define FPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fps_plan fps_plan;
typedef struct fps_batch fps_batch;

typedef enum {
  FPS_OK = 0,
  FPS_E_ARG = 1,          /* invalid argument (null pointer, n < 1, tol not in (0,1), ...) */
  FPS_E_UNSUPPORTED = 2,  /* valid but not implemented combination                      */
  FPS_E_NOMEM = 3,        /* host or device allocation failed (plan creation only)      */
  FPS_E_HIP = 4,          /* a HIP runtime call failed                                  */
  FPS_E_STATE = 5         /* plan used after destroy, or workspace too small            */
} fps_status;

typedef enum { FPS_BC_DIRICHLET_ZERO = 0 } fps_bc;

/* FPS_FP64: every ADI half-sweep stores and computes in float64.
 * FPS_FP32_REFINED: iterative refinement (precision form; not in the paper).
 * Each round forms the residual r = G - (A~ Y + Y A~) in float64, stores it
 * in float32, runs an inner ADI on A~ dY + dY A~ = r that stores every sweep
 * array (and its result dY) in float32, and adds dY to the float64 Y.  Every
 * arithmetic operation and every table stays float64.  The inner ADI applies
 * its shifts in order of increasing |p_j| (with the opposite order float
 * storage stalls or diverges from n ~ 256 on).  Rounds: inner tolerance 1e-5
 * (on smooth data a round contracts the error by about 1e-5) until one more
 * such round would pass tol, then a last round to 0.1 tol / (error
 * reached); at tol = 1e-13: 1e-5, 1e-5, 1e-4 (fps_plan_rounds).  Plans
 * created with FPS_PLAN_DIRICHLET, whose lift puts O(1) content into the
 * highest modes of G's first two rows and columns, run two float rounds
 * and then one round with float64 storage (float rounds contract such data
 * by only ~1e-3). */
typedef enum { FPS_FP64 = 0, FPS_FP32_REFINED = 1 } fps_prec;

typedef enum { FPS_OUT_CHEB = 0, FPS_OUT_NATIVE = 1 } fps_out;

/* Plan flags. */
#define FPS_PLAN_HOST_ONLY 1u  /* build host tables only (no device memory); for inspection */
/* Shift intervals from the computed extreme eigenvalues of A~ (Sturm
 * bisection, widened by a relative 1e-6) instead of the enclosure
 * [-1, -1/(30 n^4)] of Lemma B.1.  Theorem 2.1 only needs intervals that
 * contain the spectra, so the error bound and tol keep their meaning; J
 * drops (121 -> 96 at n = 4096, tol 1e-13). */
#define FPS_PLAN_TIGHT_SPECTRUM 2u
/* Cube plans: solve through the eigenbasis of A~ along z (dense MFMA
 * transforms) and one 2D ADI per z-slice, instead of the two-level nested
 * ADI.  Each slice equation (A~ + mu) Y (A~ + mu) - mu^2 Y = -G^ (mu an
 * eigenvalue of A~) is solved for Z = (A~ + mu) Y as
 * (-mu^2 (A~ + mu)^-1) Z - Z (-(A~ + mu)) = -G^ by Algorithm 2 with the slice's
 * own Zolotarev shifts; n <= 512.  Where a plan-time model predicts a gain
 * (n = 256: 78 of 256 slices), the slices with the most steps iterate on a
 * default-priority stream the plan owns, forked from and joined back to the
 * solve's stream with events, so the solve still completes in order on
 * that stream (and captures into a graph).  Solves of one plan issued on
 * several streams queue their side-stream work on that one stream, one
 * after another. */
#define FPS_PLAN_CUBE_ZEIG 4u
/* Square and rectangle plans: also build the lift map that
 * fps_solve_dirichlet needs (the scaled C~ coefficients of every T_k'', two
 * parity blocks of about (n/2)^2 float64 each: 67 MB at n = 4096) and the
 * workspace room for the lift (4 n + 8 float64). */
#define FPS_PLAN_DIRICHLET 8u

/*
 * Create a plan for a solve of size n (coefficients per dimension).
 *   dim        2 (square, Sec. 3) or 3 (cube, Sec. 5).
 *   n          >= 1; square plans n <= 16384 (chains of up to 128 chunks,
 *              the chunk-carry scan's register form), cube plans n <= 384
 *              (nested method) or n <= 512 (FPS_PLAN_CUBE_ZEIG);
 *              FPS_E_UNSUPPORTED beyond.
 *   bc         FPS_BC_DIRICHLET_ZERO (the only value).
 *   tol        0 < tol < 1; the ADI count J follows (2.9), so that the
 *              symmetrized iterate satisfies ||Y - Y_J||_2 <= tol ||Y||_2
 *              (Theorem 2.1).
 *   prec       a value of fps_prec; cube plans take FPS_FP32_REFINED with
 *              FPS_PLAN_CUBE_ZEIG only.
 *   out_basis  fps_out.
 *   flags      0 or a combination of FPS_PLAN_HOST_ONLY,
 *              FPS_PLAN_TIGHT_SPECTRUM, FPS_PLAN_CUBE_ZEIG (dim 3) and
 *              FPS_PLAN_DIRICHLET (dim 2).
 * On success *out receives a plan to release with fps_plan_destroy.
 */
fps_status fps_plan_create(fps_plan **out, int dim, int64_t n, int bc, double tol,
                           int prec, int out_basis, unsigned flags);

/*
 * Rectangle plan: u_xx + u_yy = f on [a, b] x [c, d], box_host = {a, b, c, d}
 * (host array, finite, a < b, c < d).  f, u and the boundary data are
 * expanded in the mapped variables s = (2x - a - b)/(b - a) and
 * t = (2y - c - d)/(d - c) (rows of F and U <-> t, as for the square).  The
 * symmetric form becomes sx2 A~ Y + sy2 Y A~ = G with sx2 = (2/(b-a))^2,
 * sy2 = (2/(d-c))^2 (the rectangle remark of Sec. 3, with the scalings of
 * u_ss and u_tt), i.e. A Y - Y B = G with A = sx2 A~ and B = -sy2 A~, whose
 * spectra lie in sx2 [lo, hi] and sy2 [-hi, -lo] for the enclosure [lo, hi]
 * of sigma(A~) (Lemma B.1, or the computed one with
 * FPS_PLAN_TIGHT_SPECTRUM).  Those intervals are not mirror images, so
 * Algorithm 2 runs with the general shifts (p_j, q_j) of Theorem 2.1 and two
 * shifted tridiagonal solves per step.  tol, prec, out_basis and flags as for
 * fps_plan_create (dim 2; FPS_PLAN_CUBE_ZEIG is rejected).  The plan serves
 * fps_solve, fps_solve_dirichlet, fps_solve_adjoint and fps_adi_native.
 */
fps_status fps_plan_create_rect(fps_plan **out, int64_t n, const double *box_host, double tol,
                                int prec, int out_basis, unsigned flags);

/*
 * Cylinder plan (Sec. 4.1): Poisson on x^2 + y^2 <= 1, |z| <= 1 with zero
 * Dirichlet data, through the DFS doubling (r over [-1, 1]) and a
 * Chebyshev (r) x Fourier (theta) x Chebyshev (z) expansion (4.4).
 *   n        even, 2 <= n <= 512: Chebyshev coefficients in r and in z.
 *   n_theta  even, 2 <= n_theta <= 1024: Fourier modes k = -n_theta/2 ..
 *            n_theta/2 - 1 (index k + n_theta/2).
 *   flags    0 or FPS_PLAN_HOST_ONLY.
 * fps_solve then takes F_dev = the doubled-up right-hand side as split
 * complex float64 [n_theta][2][n][n] (index 1: real, imaginary part; rows
 * <-> T_i(r), columns <-> T_j(z)) and writes U_dev [n_theta][2][n+4][n+2],
 * the Chebyshev coefficients of each mode u~_k(r, z) (r-degree up to n+3
 * from the partial-regularity factor r^min(|k|,2) (1-r^2)(1-z^2) of (4.7)).
 * Each mode solves the Galerkin system of its case of Sec. 4.1 ((4.8) for
 * |k| >= 2, the displayed operators for |k| = 1 and k = 0) exactly up to
 * rounding: in the eigenbasis of A~ along z every mode splits into banded
 * systems in r, factored by the plan (no ADI, so J = 0 and no tolerance).
 * The mode's right-hand side rows of the wrong r-parity (zero for
 * doubled-up data) are ignored.  fps_solve_adjoint, fps_adi_native and
 * fps_solve_dirichlet reject cylinder plans.
 */
fps_status fps_plan_create_cylinder(fps_plan **out, int64_t n, int64_t n_theta, unsigned flags);

/* Inspection: the band of mode k's r-operators in the parity-restricted index
 * (rows of the right-hand side parity, columns of w's parity), offsets
 * -2..2: P_host[a*5 + c], Q_host[a*5 + c] for a < n/2, the entry at column
 * a + c - 2 (host arrays of 5 n/2 doubles).  Host-only. */
fps_status fps_cylinder_mode_bands(int64_t n, int64_t k, double *P_host, double *Q_host);

/* J (ADI iterations of the outer level), workspace bytes required by
 * fps_solve / fps_solve_adjoint, and the number of float64 entries of U. */
fps_status fps_plan_info(const fps_plan *plan, int *J, int64_t *workspace_bytes,
                         int64_t *out_entries);

/* Refinement structure of a plan: the number of rounds (1 for FPS_FP64) and
 * the number of inner ADI steps, summed over the rounds, that store their
 * sweep arrays in float32 (0 for FPS_FP64).  Either pointer may be null. */
fps_status fps_plan_refinement(const fps_plan *plan, int *rounds, int *f32_steps);

/* The ADI steps and the inner tolerance of each refinement round (host
 * arrays, min(rounds, cap) entries; either may be null).  FPS_FP64 square
 * and rectangle plans have one round: J and tol.  FPS_E_STATE for cube and
 * cylinder plans. */
fps_status fps_plan_rounds(const fps_plan *plan, int *steps_host, double *tol_host, int cap);

/* Cube plans (dim = 3, nested ADI): the number of inner ADI steps of each of
 * the J outer steps (the (x, y) half-step of outer step i runs counts[i]
 * inner iterations on every z-slice).  Writes min(J, cap) entries;
 * FPS_E_STATE for square and z-eigenbasis plans. */
fps_status fps_plan_inner_counts(const fps_plan *plan, int *counts, int cap);

/* Cube plans with FPS_PLAN_CUBE_ZEIG: the number of z-slices solved (*count,
 * = n) and, if counts is non-null, the ADI steps of each slice (slices
 * sorted by decreasing count; min(*count, cap) entries).  FPS_E_STATE for
 * other plans. */
fps_status fps_plan_slice_counts(const fps_plan *plan, int *counts, int cap, int *count);

/* Copy the plan's shifts p_0..p_{J-1} to host memory, in the order the ADI
 * applies them (q_j = -p_j for the square, Sec. 3.3 P2 with B~ = -A~; for
 * the cube, the outer shifts p_i in [-2/delta, -2] of the split of (5.2)
 * into H = K_x + K_y and V = K_z, K = -A~^-1, whose partners q_i lie in
 * [1, 1/delta]).  Square and rectangle plans apply the shifts of
 * Theorem 2.1 in order of increasing |p_j|: the iterate is the same in exact
 * arithmetic, and the large-shift steps then damp the rounding that the
 * small-shift solves magnify.  FP32_REFINED plans: the shifts of round 0
 * (J = fps_plan_info's J). */
fps_status fps_plan_shifts(const fps_plan *plan, double *p_host);

/* Copy both shift sequences p_0..p_{J-1} and q_0..q_{J-1} (Theorem 2.1) to
 * host memory; for a rectangle plan they are not mirror images. */
fps_status fps_plan_shift_pairs(const fps_plan *plan, double *p_host, double *q_host);

/*
 * Shifts of Theorem 2.1 for sigma(A) in [a,b], sigma(B) in [c,d],
 * a < b < c < d, 0 < tol < 1: J from (2.9) (App. A semantics).  Writes J and,
 * if cap >= J, p[0..J-1], q[0..J-1] (host arrays of length cap).  Returns
 * FPS_E_ARG for invalid intervals or tol, FPS_E_STATE (with *J set) if
 * cap < J.  Host-only; needs no device.
 */
fps_status fps_adi_shifts(double a, double b, double c, double d, double tol, int cap,
                          int *J, double *p_host, double *q_host);

/*
 * Solve.  F_dev: n^dim float64 Chebyshev coefficients of f.  U_dev: output
 * ((n+2)^dim, or n^dim with FPS_OUT_NATIVE).  ws_dev: workspace of at least
 * fps_plan_info's workspace_bytes, 256-byte aligned.  Enqueued on `stream`;
 * returns without synchronizing.  F_dev and U_dev must not overlap ws_dev.
 * The enqueue is kernel launches only (no allocation, memset, memcpy or
 * synchronization), so it may be captured into a HIP graph for every plan
 * kind; capture with sweep timing off (fps_plan_set_sweep_timing(plan, 0)),
 * since timed launches record events.
 */
fps_status fps_solve(fps_plan *plan, const double *F_dev, double *U_dev, void *ws_dev,
                     void *stream);

/*
 * Solve with nonhomogeneous Dirichlet data (Sec. 6.1), square or rectangle
 * plans created with FPS_PLAN_DIRICHLET and FPS_OUT_CHEB (FPS_E_STATE
 * without the flag, FPS_E_UNSUPPORTED for other plans).  bc_dev: 4 x (n+2) float64, rows L, R, B, T = the
 * Chebyshev coefficients of u(a, y) and u(b, y) in t, and of u(x, c) and
 * u(x, d) in s ([-1, 1]^2 for a square plan).  The corners should agree
 * (L(-1) = B(-1), L(1) = T(-1), R(-1) = B(1), R(1) = T(1)); the lift's
 * bilinear corner term takes its values from B and T.  U = U_0 + U_bc with
 * U_bc the Chebyshev coefficients of the transfinite interpolant
 * u_bc = (1-s)/2 L + (1+s)/2 R + (1-t)/2 B + (1+t)/2 T - bilinear corners,
 * and U_0 the zero-data solution for f - Lap u_bc (the C~ projection of
 * Lap u_bc enters G; it touches only two rows and two columns, and is formed
 * from the traces by the plan's lift map, which maps Chebyshev coefficients
 * straight to C~ coefficients of the second derivative: forming g'' first
 * and projecting it cancels by up to ~4e3 for rough traces).  Workspace,
 * stream and overlap rules as for fps_solve; bc_dev must not overlap ws_dev.
 */
fps_status fps_solve_dirichlet(fps_plan *plan, const double *F_dev, const double *bc_dev,
                               double *U_dev, void *ws_dev, void *stream);

/*
 * Adjoint (vector-Jacobian product) of fps_solve: given Ubar (same layout as
 * U) returns Fbar (n^dim) with <U(F), Ubar> = <F, Fbar> for the J-step ADI
 * map.  The symmetric-shift ADI map is self-adjoint in the Frobenius inner
 * product (every term is phi(A~) G psi(A~) with symmetric phi, psi), so the
 * adjoint runs the same sweeps between transposed coefficient maps.  The
 * same holds for a rectangle plan's general shifts: the J-step error map is
 * r(A) E r(B)^-1 with r a rational function and A, B symmetric, so the map
 * is a multiplier in the orthonormal eigenbasis of A~.
 * Square and rectangle plans (dim = 2), FPS_FP64 only.
 */
fps_status fps_solve_adjoint(fps_plan *plan, const double *Ubar_dev, double *Fbar_dev,
                             void *ws_dev, void *stream);

/*
 * Stage entry point of the square solve, for testing the ADI sweeps on their
 * own: G_dev (n x n, natural index order) is the right-hand side of the
 * symmetric form A~ Y + Y A~ = G of (3.9); Y_dev (n x n) receives the J-step
 * iterate Y_J of Algorithm 2 (A = A~, B = -A~, q_j = -p_j, X_0 = 0).  For a
 * rectangle plan the equation is sx2 A~ Y + sy2 Y A~ = G with the plan's
 * (p_j, q_j).  2-D plans; uses the same workspace as fps_solve.
 */
fps_status fps_adi_native(fps_plan *plan, const double *G_dev, double *Y_dev, void *ws_dev,
                          void *stream);

/*
 * Diagnostics for throughput measurement.  fps_plan_set_sweep_timing(plan,
 * capacity) creates `capacity` HIP event pairs (0 disables and releases
 * them); later solves time each ADI half-sweep launch with one pair (the
 * dispatch's own start and end timestamps), until the pairs run out.
 * fps_plan_sweep_time waits for the recorded events, writes the elapsed
 * milliseconds of the timed launches in launch order to
 * ms_host[0..min(count, cap)-1] (ms_host may be null when cap is 0), sets
 * *launches to their count, and resets the count.  Square plans: half-step 1
 * and half-step 2 of Algorithm 2 alternate, starting with half-step 1; cube
 * plans: per outer step one z sweep, then the inner half-steps 1 and 2;
 * z-eigenbasis cube plans: per step j the x solves of all slices still
 * iterating, then their y solves (one launch each).
 */
fps_status fps_plan_set_sweep_timing(fps_plan *plan, int capacity);
fps_status fps_plan_sweep_time(fps_plan *plan, double *ms_host, int64_t cap, int64_t *launches);

/*
 * Allocation-free solve, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): fps_solve with the workspace taken from a static device array
 * of fps_noalloc_capacity() bytes (64 MiB) that the library holds on every
 * GPU it runs on until the process ends.  The caller passes F_dev and U_dev
 * as for fps_solve; nothing is allocated or freed (no hipMalloc, no library
 * allocator).  Square and rectangle plans (dim 2) whose workspace_bytes fit
 * the array: FP64 up to about n = 1150, FPS_FP32_REFINED up to about
 * n = 1100.  Larger plans, cube and cylinder plans return FPS_E_UNSUPPORTED
 * with the sizes in fps_last_error().  Every call on one GPU shares that
 * GPU's array, and the solve reads only what it wrote in the same call:
 * calls that overlap on one GPU (two streams, or two host threads) race and
 * give wrong results; calls in stream order do not.  The first call on a
 * device looks up the array's device address (hipGetSymbolAddress).
 */
int64_t fps_noalloc_capacity(void);
fps_status fps_solve_noalloc(fps_plan *plan, const double *F_dev, double *U_dev, void *stream);

/*
 * Measurement aid, not part of the solver: c[i] = a[i] + b[i] for i < n, a
 * pure streaming pass (two reads and one write of 8 bytes per element, in
 * 16-byte accesses) whose rate on arrays far larger than the last-level
 * cache is the HBM rate a kernel of the sweeps' access pattern can reach.
 * a, b, c: device arrays of n doubles, 16-byte aligned, c not overlapping a
 * or b; n >= 0 (n = 0 does nothing).  Enqueued on `stream`; FPS_E_ARG for a
 * null or misaligned array or n < 0.
 */
fps_status fps_probe_stream(const double *a, const double *b, double *c, int64_t n, void *stream);

void fps_plan_destroy(fps_plan *plan);

/*
 * Batched square solves (a batching form of the same solve; not in the
 * paper): `count` independent problems of sizes n[0..count-1], each solved
 * exactly as fps_solve with a plan of that size, tol, precision and output
 * basis would solve it.  Problems of equal n share one set of plan tables.
 * The ADI half-sweeps of all problems run as one launch per half-step (the
 * problems still iterating at that step), so a batch enqueues about 4 J_max
 * sweep/carry launches plus a fixed number of map launches per problem.
 *   dim must be 2; 1 <= count <= 65536; every n in [1, 16384]; tol, prec,
 *   out_basis and flags as for fps_plan_create.  FPS_FP32_REFINED batches
 *   run the rounds of their plans (the same round tolerances for every
 *   problem), one batched inner ADI per round.
 * Data: F_dev packs the problems' n x n inputs back to back in the given
 * order (row-major each, offsets sum of n_b^2); U_dev packs the outputs
 * ((n_b+2)^2 or n_b^2 entries each).  fps_batch_info gives the totals and the
 * workspace size; the workspace must be 256-byte aligned and must not
 * overlap F or U.  fps_batch_solve enqueues on `stream` without allocating
 * or synchronizing and without memset or memcpy nodes, so it may be captured
 * into a HIP graph.
 */
fps_status fps_batch_create(fps_batch **out, int dim, int count, const int64_t *n, double tol,
                            int prec, int out_basis, unsigned flags);
fps_status fps_batch_info(const fps_batch *batch, int64_t *workspace_bytes, int64_t *in_entries,
                          int64_t *out_entries, int *max_J);
fps_status fps_batch_solve(fps_batch *batch, const double *F_dev, double *U_dev, void *ws_dev,
                           void *stream);
/* Adjoint (vector-Jacobian product) of fps_batch_solve, the batched form of
 * fps_solve_adjoint: Ubar_dev in the batch's output layout, Fbar_dev
 * (written) in its input layout.  Each problem's symmetric-shift ADI map of
 * Algorithm 2 (shifts of Theorem 2.1) is self-adjoint in the Frobenius inner
 * product (derived here: every term is phi(A~) G psi(A~) with symmetric
 * phi, psi), so the adjoint runs the same batched sweeps
 * between the transposed coefficient maps; every problem's result equals
 * fps_solve_adjoint on that problem.  FP64 batches only (FPS_E_UNSUPPORTED
 * otherwise); same workspace and stream rules as fps_batch_solve. */
fps_status fps_batch_solve_adjoint(fps_batch *batch, const double *Ubar_dev, double *Fbar_dev,
                                   void *ws_dev, void *stream);
void fps_batch_destroy(fps_batch *batch);

const char *fps_status_string(fps_status s);
const char *fps_last_error(void);
const char *fps_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FPS_H */
