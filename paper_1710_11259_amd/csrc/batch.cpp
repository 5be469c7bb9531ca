// Batched square solves (fps_batch_* in include/fps.h): many independent
// problems, possibly of different sizes, whose ADI half-sweeps run as one
// launch per half-step.  Every problem keeps the tables, workspace layout,
// shifts and kernels of its own single-problem plan; only the launch of the
// sweeps and of the chunk-carry reductions is shared.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <new>
#include <numeric>
#include <vector>

#include "launch_limits.hpp"
#include "solver.hpp"

using namespace fps::detail;

namespace {

constexpr uint64_t kBatchMagic = 0x66707362'61746331ull;  // "fpsbatc1"

}  // namespace

struct fps_batch {
  uint64_t magic = kBatchMagic;
  int count = 0, prec = FPS_FP64, out_basis = FPS_OUT_CHEB;
  bool on_device = false;
  std::vector<int64_t> n;            // per problem, caller's order
  std::vector<fps_plan *> sub;       // one plan per distinct n (owned)
  std::vector<int> which;            // problem -> index into sub
  std::vector<int> order;            // sorted position -> problem (J descending)
  std::vector<int64_t> f_off, u_off, ws_off;  // per problem: F / U entries, workspace bytes
  int64_t in_entries = 0, out_entries = 0, ws_bytes = 0;
  int J_max = 0;                     // steps of the longest ADI (over all rounds)
  // Refinement rounds (1 for FP64; the storage type of each round is its
  // plans' rf32[r]).  Round r has J_r[r] steps at most; at its step j the
  // problems still iterating are the sorted prefix active[r][j]; its
  // descriptors start at step row row0[r] of the sweep / carry tables.
  int rounds = 1;
  std::vector<int> J_r, row0;
  std::vector<std::vector<int>> active;
  std::vector<int> sw_start, rd_start;  // workgroup prefix sums over the sorted problems
  int64_t ncmax_max = 0;
  DeviceBuf d_sw, d_rd, d_swmap, d_rdmap;
  // coefficient-map GEMMs of all problems: input map g1, g2; output map g1,
  // g2; (FP64 batches) the adjoint's input map g1, g2 and output map g1, g2
  DeviceBuf d_gd[8], d_gmap[8];
  int gtiles[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // permute-in (0), 64 x 64 tiles (1: the map and descriptors the refined
  // residual launch runs on), finalize (2) and, for refined batches,
  // residual (3) of all problems as one launch each (elem_ok; else, for very
  // large batches, one launch per problem)
  bool elem_ok = false;
  DeviceBuf d_ed[4], d_emap[3];
  int ewg[3] = {0, 0, 0};

  ~fps_batch() {
    for (fps_plan *p : sub) fps_plan_destroy(p);
  }
  const fps_plan *plan_of(int problem) const { return sub[which[problem]]; }
};

namespace {

bool valid_batch(const fps_batch *b) { return b != nullptr && b->magic == kBatchMagic; }

// Byte offset carried in a descriptor's pointer field.
template <typename P>
P off_ptr(int64_t off) {
  return (P)(intptr_t)off;
}

// GEMM tables of the coefficient maps: the single-problem builders run on
// synthetic base pointers (the problem's workspace offset, its U offset in
// bytes), so every workspace or output operand comes out as an offset.
fps_status build_gemm_tables(fps_batch *bt) {
  std::vector<fps::GemmDesc> tab[8];
  const bool refined = bt->prec == FPS_FP32_REFINED;
  for (int b = 0; b < bt->count; ++b) {
    const fps_plan *pl = bt->plan_of(b);
    char *wsyn = (char *)(intptr_t)bt->ws_off[b];
    fps::GemmProb g[8][4];
    const int c_in = rhs_gemms(pl, wsyn, g[0], g[1]);
    const double *Ysyn = (const double *)(wsyn + (refined ? pl->off_GT : pl->off_G));
    double *Usyn = (double *)(intptr_t)(bt->u_off[b] * (int64_t)sizeof(double));
    const bool cheb = bt->out_basis == FPS_OUT_CHEB;
    const int c_out = cheb ? out_gemms(pl, Ysyn, Usyn, wsyn, g[2], g[3]) : 0;
    // adjoint (FP64): Ubar -> Ybar (Chebyshev output), Gbar (in G) -> Fbar,
    // Fbar as an offset into the input layout
    int c_ain = 0, c_aout = 0;
    if (!refined) {
      c_ain = cheb ? adj_in_gemms(pl, wsyn, g[4], g[5]) : 0;
      double *Fsyn = (double *)(intptr_t)(bt->f_off[b] * (int64_t)sizeof(double));
      c_aout = adj_out_gemms(pl, (const double *)(wsyn + pl->off_G), Fsyn, wsyn, g[6], g[7]);
    }
    // base ids (A, B, C): ws-relative 1, absolute 0, output-relative 2
    static const int ids[8][3] = {{1, 0, 1}, {0, 1, 1}, {1, 0, 1}, {0, 1, 2},
                                  {1, 0, 1}, {0, 1, 1}, {1, 0, 1}, {0, 1, 2}};
    const int counts[8] = {c_in, c_in, c_out, c_out, c_ain, c_ain, c_aout, c_aout};
    for (int t = 0; t < 8; ++t) {
      const int cnt = counts[t];
      for (int i = 0; i < cnt; ++i) {
        if (!fps::gemm_operands_ok(g[t][i]))
          return fail(FPS_E_STATE, "internal: batched GEMM operand layout");
        fps::GemmDesc d{g[t][i], ids[t][0], ids[t][1], ids[t][2], bt->gtiles[t], 0};
        bt->gtiles[t] += fps::gemm_tiles(g[t][i], &d.ntx);
        tab[t].push_back(d);
      }
    }
  }
  for (int t = 0; t < 8; ++t) {
    if (tab[t].empty()) continue;
    const std::vector<int> map = fps::gemm_table_map(tab[t]);
    fps_status s;
    if ((s = upload(bt->d_gd[t], tab[t])) != FPS_OK || (s = upload(bt->d_gmap[t], map)) != FPS_OK)
      return s;
  }
  return FPS_OK;
}

fps_status build_elem_tables(fps_batch *bt);

// Builds the per-step descriptors of every problem (sorted order) and the
// workgroup -> problem maps.
fps_status build_descriptors(fps_batch *bt) {
  const int C = bt->count;
  const bool refined = bt->prec == FPS_FP32_REFINED;
  const int gf = refined ? 1 : 0;
  const int rows = bt->row0.back() + bt->J_r.back();
  std::vector<fps::BatchSweep> sw((size_t)rows * 2 * C);
  std::vector<fps::BatchReduce> rd((size_t)rows * 2 * C);
  for (int k = 0; k < C; ++k) {
    const int b = bt->order[k];
    const fps_plan *pl = bt->plan_of(b);
    const fps::Layout &L = pl->L;
    const int64_t W = bt->ws_off[b];
    const int64_t Gterm = W + (refined ? pl->off_R : pl->off_G);
    const int64_t O0 = W + pl->off_O0, O1 = W + pl->off_O1, lv = W + pl->off_lv,
                  ab = W + pl->off_ab;
    fps::SweepArgs A{};
    A.npad = L.npad;
    A.ncols = L.npad;
    A.ld = L.npad;
    A.nbatch = 1;
    A.mp0 = L.mp[0];
    A.mp1 = L.mp[1];
    A.mstride = L.mstride;
    A.ncmax = L.ncmax;
    A.nc0 = (int)L.nc[0];
    A.nc1 = (int)L.nc[1];
    A.lv = off_ptr<double *>(lv);
    const int nbx_s = (int)(L.npad / fps::kCols);
    const int rchains = fps::reduce_chains(bt->ncmax_max);
    const int nbx_r = (int)((L.npad + rchains - 1) / rchains);
    for (int r = 0; r < bt->rounds; ++r) {
      const fps::ShiftSet &sh = pl->rsh[(size_t)r];
      const int J = sh.J, base = pl->rbase[(size_t)r];
      const int f = pl->rf32[(size_t)r];
      const std::vector<double> &p = sh.p;
      for (int j = 0; j < J; ++j) {
        const bool last = j == J - 1;
        // half-step 1: row chains, output in the input's layout
        fps::SweepArgs a1 = A;
        a1.in = off_ptr<const void *>(j == 0 ? Gterm : O1);
        a1.in_f32 = j == 0 ? gf : f;
        a1.in_scale = j == 0 ? -1.0 : 1.0;
        a1.ab_prev = j == 0 ? nullptr : off_ptr<const double *>(ab);
        a1.tab_prev = j == 0 ? nullptr : pl->tab_dev(base + j - 1);
        a1.g = nullptr;
        a1.tab = pl->tab_dev(base + j);
        a1.l1 = pl->l1_dev(base + j);
        a1.sigma = 2.0 * p[j];
        a1.out = off_ptr<void *>(O0);
        a1.out_f32 = f;
        a1.out_mode = 0;
        // half-step 2: column chains, stored in place
        fps::SweepArgs a2 = a1;
        a2.in = off_ptr<const void *>(O0);
        a2.in_f32 = f;
        a2.in_scale = 1.0;
        a2.ab_prev = off_ptr<const double *>(ab);
        a2.tab_prev = pl->tab_dev(base + j);
        a2.g = off_ptr<const void *>(Gterm);
        a2.g_f32 = gf;
        a2.sg = 1.0;
        a2.sigma = last ? 0.0 : p[j] + p[j + 1];
        a2.out = off_ptr<void *>(O1);
        a2.out_f32 = f;
        a2.out_mode = last ? 1 : 2;
        const int row = bt->row0[(size_t)r] + j;
        const size_t i1 = ((size_t)row * 2 + 0) * C + k, i2 = ((size_t)row * 2 + 1) * C + k;
        sw[i1] = fps::BatchSweep{a1, bt->sw_start[k], nbx_s};
        sw[i2] = fps::BatchSweep{a2, bt->sw_start[k], nbx_s};
        rd[i1] = fps::BatchReduce{lv, ab, pl->ctab_dev(base + j), -a1.sigma, L.npad, L.ncmax,
                                  (int)L.nc[0], (int)L.nc[1], bt->rd_start[k], nbx_r};
        rd[i2] = rd[i1];
        rd[i2].scale = last ? 1.0 : -a2.sigma;
      }
    }
  }
  std::vector<int> swmap(bt->sw_start[C]), rdmap(bt->rd_start[C]);
  for (int k = 0; k < C; ++k) {
    std::fill(swmap.begin() + bt->sw_start[k], swmap.begin() + bt->sw_start[k + 1], k);
    std::fill(rdmap.begin() + bt->rd_start[k], rdmap.begin() + bt->rd_start[k + 1], k);
  }
  fps_status s;
  if ((s = upload(bt->d_sw, sw)) != FPS_OK || (s = upload(bt->d_rd, rd)) != FPS_OK ||
      (s = upload(bt->d_swmap, swmap)) != FPS_OK || (s = upload(bt->d_rdmap, rdmap)) != FPS_OK)
    return s;
  if ((s = build_gemm_tables(bt)) != FPS_OK) return s;
  return build_elem_tables(bt);
}

// Tables of the batched element-wise launches (sorted order, largest
// problems first).  Left unbuilt (elem_ok false) when a launch would not fit
// one 1-D grid of 256-thread workgroups (elem_launch_fits); such batches
// keep the per-problem launches.

fps_status build_elem_tables(fps_batch *bt) {
  const int C = bt->count;
  const bool refined = bt->prec == FPS_FP32_REFINED;
  std::vector<fps::ElemDesc> ed[4];
  int64_t tot[3] = {0, 0, 0};
  for (int k = 0; k < C; ++k) {
    const int b = bt->order[k];
    const fps_plan *pl = bt->plan_of(b);
    const fps::Layout &L = pl->L;
    const int64_t W = bt->ws_off[b], rowb = (L.npad + 255) / 256, tb = L.npad / 64;
    const int64_t nwg[3] = {rowb * L.npad, tb * tb, rowb * L.npad};
    for (int t = 0; t < 3; ++t)
      if (!fps::elem_launch_fits(tot[t] + nwg[t])) return FPS_OK;  // elem_ok stays false
    fps::ElemDesc e{};
    e.n = L.n;
    e.npad = L.npad;
    e.mp0 = L.mp[0];
    e.mstride = L.mstride;
    e.ncmax = L.ncmax;
    e.sbase = e.dbase = 1;
    fps::ElemDesc pin = e;  // F -> the G^T region
    pin.src = bt->f_off[b] * (int64_t)sizeof(double);
    pin.sbase = 2;
    pin.dst = W + pl->off_GT;
    pin.nbx = (int)rowb;
    fps::ElemDesc tr = e;  // 64 x 64 tiles: the workgroup map of the residual
    tr.nbx = (int)tb;
    fps::ElemDesc fin = e;  // O1 and its carries -> Y (round 0's tables)
    fin.src = W + pl->off_O1;
    fin.ab = W + pl->off_ab;
    fin.tab = pl->tab_dev(pl->rbase[0] + pl->rsh[0].J - 1);
    fin.dst = W + (refined ? pl->off_GT : pl->off_G);
    fin.nbx = (int)rowb;
    fps::ElemDesc *all[3] = {&pin, &tr, &fin};
    for (int t = 0; t < 3; ++t) {
      all[t]->wg_start = (int)tot[t];
      tot[t] += nwg[t];
      ed[t].push_back(*all[t]);
    }
    if (refined) {  // r = G - (A~ Y + Y A~) into the float residual region
      fps::ElemDesc res = tr;
      res.src = W + pl->off_G;
      res.ab = W + pl->off_GT;
      res.dst = W + pl->off_R;
      res.tab = (const double *)pl->d_sdiag.p;
      res.ev = (const double *)pl->d_soff.p;
      ed[3].push_back(res);
    }
  }
  fps_status s;
  for (int t = 0; t < 3; ++t) {
    std::vector<int> map((size_t)tot[t]);
    for (int k = 0; k < C; ++k) {
      const int64_t lo = ed[t][(size_t)k].wg_start;
      const int64_t hi = k + 1 < C ? ed[t][(size_t)k + 1].wg_start : tot[t];
      std::fill(map.begin() + lo, map.begin() + hi, k);
    }
    if ((s = upload(bt->d_ed[t], ed[t])) != FPS_OK || (s = upload(bt->d_emap[t], map)) != FPS_OK)
      return s;
    bt->ewg[t] = (int)tot[t];
  }
  if (refined && (s = upload(bt->d_ed[3], ed[3])) != FPS_OK) return s;
  // The finalize descriptors of the later refinement rounds (the tables of
  // each round's last step; same workgroup map).
  if (bt->rounds > 1) {
    std::vector<fps::ElemDesc> fr;
    for (int r = 0; r < bt->rounds; ++r)
      for (int k = 0; k < C; ++k) {
        fps::ElemDesc f = ed[2][(size_t)k];
        const fps_plan *pl = bt->plan_of(bt->order[k]);
        f.tab = pl->tab_dev(pl->rbase[(size_t)r] + pl->rsh[(size_t)r].J - 1);
        fr.push_back(f);
      }
    bt->d_ed[2].~DeviceBuf();
    new (&bt->d_ed[2]) DeviceBuf();
    if ((s = upload(bt->d_ed[2], fr)) != FPS_OK) return s;
  }
  bt->elem_ok = true;
  return FPS_OK;
}

// Final pass of every problem into Y (its G region, or G^T for a refined
// batch) after refinement round `round`: mode 0 stores, mode 2 adds.
hipError_t finalize_all(const fps_batch *bt, char *w, int mode, int round, hipStream_t st) {
  if (bt->elem_ok)
    return fps::launch_finalize_batch((const fps::ElemDesc *)bt->d_ed[2].p + (size_t)round * bt->count,
                                      (const int *)bt->d_emap[2].p, bt->ewg[2], mode, w, st,
                                      bt->sub[0]->rf32[(size_t)round]);
  const bool refined = bt->prec == FPS_FP32_REFINED;
  const bool xf = bt->sub[0]->rf32[(size_t)round] != 0;
  for (int b = 0; b < bt->count; ++b) {
    const fps_plan *pl = bt->plan_of(b);
    const fps::Layout &L = pl->L;
    char *wb = w + bt->ws_off[b];
    double *Y = (double *)(wb + (refined ? pl->off_GT : pl->off_G));
    const double *tab = pl->tab_dev(pl->rbase[(size_t)round] + pl->rsh[(size_t)round].J - 1);
    const double *ab = (const double *)(wb + pl->off_ab);
    const hipError_t e =
        xf ? fps::launch_finalize<float>((const float *)(wb + pl->off_O1), ab, tab, Y, mode,
                                              nullptr, L.n, L.npad, L.mp[0], L.mstride, L.ncmax, st)
                : fps::launch_finalize<double>((const double *)(wb + pl->off_O1), ab, tab, Y, mode,
                                               nullptr, L.n, L.npad, L.mp[0], L.mstride, L.ncmax,
                                               st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The batched half-steps of refinement round `round` (and their carry
// reductions).  At step j the problems with J > j form a prefix of the
// sorted order; a problem's last step writes its final chunk-local solution
// to its O1 and its carries to its ab, which later steps leave alone.
fps_status run_adi_batch(fps_batch *bt, int round, char *ws, hipStream_t st) {
  const int C = bt->count;
  const int f = bt->sub[0]->rf32[(size_t)round];
  const int gf = bt->prec == FPS_FP32_REFINED ? 1 : 0;  // the residual r is stored in float
  const fps::BatchSweep *dsw = (const fps::BatchSweep *)bt->d_sw.p;
  const fps::BatchReduce *drd = (const fps::BatchReduce *)bt->d_rd.p;
  const int *swmap = (const int *)bt->d_swmap.p, *rdmap = (const int *)bt->d_rdmap.p;
  const std::vector<int> &act = bt->active[(size_t)round];
  for (int j = 0; j < bt->J_r[(size_t)round]; ++j) {
    const int k = act[(size_t)j];
    // the storage types of every descriptor of the launch (a problem's last
    // step writes double, and its later steps are not launched)
    fps::SweepArgs t1{};
    t1.in_f32 = j == 0 ? gf : f;
    t1.out_f32 = f;
    fps::SweepArgs t2{};
    t2.in_f32 = f;
    t2.g_f32 = gf;
    t2.out_f32 = f;
    const int row = bt->row0[(size_t)round] + j;
    const size_t o1 = ((size_t)row * 2 + 0) * C, o2 = ((size_t)row * 2 + 1) * C;
    FPS_HIP(fps::launch_sweep_batch_rows(t1, dsw + o1, swmap, bt->sw_start[k], ws, st));
    FPS_HIP(fps::launch_reduce_batch(drd + o1, rdmap, bt->rd_start[k], bt->ncmax_max, ws, st));
    FPS_HIP(fps::launch_sweep_batch(t2, true, dsw + o2, swmap, bt->sw_start[k], ws, st));
    FPS_HIP(fps::launch_reduce_batch(drd + o2, rdmap, bt->rd_start[k], bt->ncmax_max, ws, st));
  }
  return FPS_OK;
}

}  // namespace

extern "C" {

fps_status fps_batch_create(fps_batch **out, int dim, int count, const int64_t *n, double tol,
                            int prec, int out_basis, unsigned flags) {
  if (!out) return fail(FPS_E_ARG, "out must not be null");
  *out = nullptr;
  if (dim == 3) return fail(FPS_E_UNSUPPORTED, "batched solves are square only");
  if (dim != 2) return fail(FPS_E_ARG, "dim must be 2 or 3");
  if (count < 1 || count > 65536) return fail(FPS_E_ARG, "count must lie in [1, 65536]");
  if (!n) return fail(FPS_E_ARG, "n must not be null");
  for (int b = 0; b < count; ++b)
    if (n[b] < 1 || n[b] > 16384) return fail(FPS_E_ARG, "every n must lie in [1, 16384]");
  fps_batch *bt = new (std::nothrow) fps_batch();
  if (!bt) return fail(FPS_E_NOMEM, "batch allocation failed");
  bt->count = count;
  bt->prec = prec;
  bt->out_basis = out_basis;
  bt->n.assign(n, n + count);
  std::map<int64_t, int> idx;
  bt->which.resize(count);
  for (int b = 0; b < count; ++b) {
    auto it = idx.find(n[b]);
    if (it == idx.end()) {
      fps_plan *pl = nullptr;
      fps_status s = fps_plan_create(&pl, 2, n[b], FPS_BC_DIRICHLET_ZERO, tol, prec, out_basis, flags);
      if (s != FPS_OK) {
        delete bt;
        return s;
      }
      it = idx.emplace(n[b], (int)bt->sub.size()).first;
      bt->sub.push_back(pl);
    }
    bt->which[b] = it->second;
  }
  bt->f_off.resize(count);
  bt->u_off.resize(count);
  bt->ws_off.resize(count);
  for (int b = 0; b < count; ++b) {
    const fps_plan *pl = bt->plan_of(b);
    bt->f_off[b] = bt->in_entries;
    bt->u_off[b] = bt->out_entries;
    bt->ws_off[b] = bt->ws_bytes;
    const int64_t e = out_basis == FPS_OUT_NATIVE ? n[b] : n[b] + 2;
    bt->in_entries += n[b] * n[b];
    bt->out_entries += e * e;
    bt->ws_bytes += align256(pl->ws_bytes);
  }
  bt->order.resize(count);
  std::iota(bt->order.begin(), bt->order.end(), 0);
  std::stable_sort(bt->order.begin(), bt->order.end(), [&](int a, int c) {
    const int Ja = bt->plan_of(a)->shifts.J, Jc = bt->plan_of(c)->shifts.J;
    return Ja != Jc ? Ja > Jc : n[a] > n[c];
  });
  // Every plan of the batch has the same round structure (the schedule
  // depends on tol only); within a round J grows with n, so the problems
  // still iterating at any step form a prefix of the sorted order.
  bt->rounds = bt->sub[0]->rounds;
  bt->J_r.assign(bt->rounds, 0);
  bt->row0.assign(bt->rounds, 0);
  bt->active.assign(bt->rounds, std::vector<int>());
  for (int r = 0; r < bt->rounds; ++r) {
    int prev = 1 << 30;
    for (int k = 0; k < count; ++k) {
      const fps_plan *pl = bt->plan_of(bt->order[k]);
      const int J = (int)pl->rsh.size() == bt->rounds ? pl->rsh[(size_t)r].J : -1;
      if (J < 0 || J > prev) {
        delete bt;
        return fail(FPS_E_STATE, "internal: batch round structure");
      }
      prev = J;
      bt->J_r[(size_t)r] = std::max(bt->J_r[(size_t)r], J);
    }
    bt->active[(size_t)r].assign(bt->J_r[(size_t)r], 0);
    for (int j = 0; j < bt->J_r[(size_t)r]; ++j)
      for (int k = 0; k < count; ++k)
        if (bt->plan_of(bt->order[k])->rsh[(size_t)r].J > j) bt->active[(size_t)r][j] = k + 1;
    if (r > 0) bt->row0[(size_t)r] = bt->row0[(size_t)r - 1] + bt->J_r[(size_t)r - 1];
    bt->J_max = std::max(bt->J_max, bt->J_r[(size_t)r]);
  }
  bt->sw_start.assign(count + 1, 0);
  bt->rd_start.assign(count + 1, 0);
  for (int k = 0; k < count; ++k)
    bt->ncmax_max = std::max(bt->ncmax_max, bt->plan_of(bt->order[k])->L.ncmax);
  const int rchains = fps::reduce_chains(bt->ncmax_max);  // chains per carry workgroup
  for (int k = 0; k < count; ++k) {
    const fps::Layout &L = bt->plan_of(bt->order[k])->L;
    const int64_t nsw = (L.npad / fps::kCols) * (L.nc[0] + L.nc[1]);
    const int64_t nrd = ((L.npad + rchains - 1) / rchains) * 2;
    if ((int64_t)bt->sw_start[k] + nsw > (int64_t)1 << 30 ||
        (int64_t)bt->rd_start[k] + nrd > (int64_t)1 << 30) {
      delete bt;
      return fail(FPS_E_UNSUPPORTED, "batch too large for one launch");
    }
    bt->sw_start[k + 1] = bt->sw_start[k] + (int)nsw;
    bt->rd_start[k + 1] = bt->rd_start[k] + (int)nrd;
  }
  if (!(flags & FPS_PLAN_HOST_ONLY)) {
    fps_status s = build_descriptors(bt);
    if (s != FPS_OK) {
      delete bt;
      return s;
    }
    bt->on_device = true;
  }
  *out = bt;
  return FPS_OK;
}

fps_status fps_batch_info(const fps_batch *bt, int64_t *ws_bytes, int64_t *in_entries,
                          int64_t *out_entries, int *max_J) {
  if (!valid_batch(bt)) return fail(FPS_E_STATE, "invalid or destroyed batch");
  if (ws_bytes) *ws_bytes = bt->ws_bytes;
  if (in_entries) *in_entries = bt->in_entries;
  if (out_entries) *out_entries = bt->out_entries;
  if (max_J) *max_J = bt->J_max;
  return FPS_OK;
}

fps_status fps_batch_solve(fps_batch *bt, const double *F, double *U, void *ws, void *stream) {
  if (!valid_batch(bt)) return fail(FPS_E_STATE, "invalid or destroyed batch");
  if (!bt->on_device) return fail(FPS_E_STATE, "batch was created host-only");
  if (!F || !U || !ws) return fail(FPS_E_ARG, "null pointer argument");
  if (((uintptr_t)ws) % 256 != 0) return fail(FPS_E_ARG, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  const int C = bt->count;
  fps_status s;
  auto gemm = [&](int t) {
    return fps::launch_gemm_table((const fps::GemmDesc *)bt->d_gd[t].p,
                                  (const int *)bt->d_gmap[t].p, bt->gtiles[t], w, (char *)U, st);
  };
  // Input maps: F into each problem's GT region, then the two GEMM stages of
  // all problems (G in its G region).
  if (bt->elem_ok)
    FPS_HIP(fps::launch_permute_in_batch((const fps::ElemDesc *)bt->d_ed[0].p,
                                         (const int *)bt->d_emap[0].p, bt->ewg[0], F, w, st));
  else
    for (int b = 0; b < C; ++b) {
      const fps_plan *pl = bt->plan_of(b);
      FPS_HIP(fps::launch_permute_in(F + bt->f_off[b], (double *)(w + bt->ws_off[b] + pl->off_GT),
                                     pl->L.n, pl->L.npad, pl->L.mp[0], st));
    }
  FPS_HIP(gemm(0));
  FPS_HIP(gemm(1));
  // Y of every problem: FP64 lands in its G region, refined in its GT region
  // (as the single-problem solve places it).
  const bool refined = bt->prec == FPS_FP32_REFINED;
  for (int k = 0; k < bt->rounds; ++k) {
    if (refined && bt->elem_ok)
      FPS_HIP(fps::launch_residual_batch((const fps::ElemDesc *)bt->d_ed[3].p,
                                         (const int *)bt->d_emap[1].p, bt->ewg[1], k != 0, w, st));
    else if (refined)
      for (int b = 0; b < C; ++b) {
        fps_plan *pl = bt->sub[bt->which[b]];
        char *wb = w + bt->ws_off[b];
        float *r = (float *)(wb + pl->off_R);
        FPS_HIP(fps::launch_residual((const double *)(wb + pl->off_G),
                                     k == 0 ? nullptr : (const double *)(wb + pl->off_GT),
                                     (const double *)pl->d_sdiag.p, (const double *)pl->d_soff.p,
                                     r, nullptr, pl->L.npad, st));
      }
    if ((s = run_adi_batch(bt, k, w, st)) != FPS_OK) return s;
    FPS_HIP(finalize_all(bt, w, k == 0 ? 0 : 2, k, st));
  }
  if (bt->out_basis == FPS_OUT_NATIVE) {
    for (int b = 0; b < C; ++b) {
      fps_plan *pl = bt->sub[bt->which[b]];
      const fps::Layout &L = pl->L;
      const double *Y = (const double *)(w + bt->ws_off[b] + (refined ? pl->off_GT : pl->off_G));
      FPS_HIP(fps::launch_permute_out(Y, U + bt->u_off[b], L.n, L.npad, L.mp[0],
                                      (const double *)pl->d_sinv.p, st));
    }
    return FPS_OK;
  }
  FPS_HIP(fps::launch_fill(U, bt->out_entries, 0.0, st));
  FPS_HIP(gemm(2));
  FPS_HIP(gemm(3));
  return FPS_OK;
}

fps_status fps_batch_solve_adjoint(fps_batch *bt, const double *Ubar, double *Fbar, void *ws,
                                   void *stream) {
  if (!valid_batch(bt)) return fail(FPS_E_STATE, "invalid or destroyed batch");
  if (!bt->on_device) return fail(FPS_E_STATE, "batch was created host-only");
  if (!Ubar || !Fbar || !ws) return fail(FPS_E_ARG, "null pointer argument");
  if (((uintptr_t)ws) % 256 != 0) return fail(FPS_E_ARG, "workspace must be 256-byte aligned");
  if (bt->prec != FPS_FP64) return fail(FPS_E_UNSUPPORTED, "batched adjoint: FP64 batches only");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  const int C = bt->count;
  fps_status s;
  auto gemm = [&](int t, char *out) {
    return fps::launch_gemm_table((const fps::GemmDesc *)bt->d_gd[t].p,
                                  (const int *)bt->d_gmap[t].p, bt->gtiles[t], w, out, st);
  };
  // Ybar of every problem into its G region: the permutations and the
  // input-map GEMMs of all problems (two table launches).
  for (int b = 0; b < C; ++b)
    if ((s = fps::detail::adjoint_in_pre(bt->plan_of(b), Ubar + bt->u_off[b], w + bt->ws_off[b],
                                         st)) != FPS_OK)
      return s;
  FPS_HIP(gemm(4, nullptr));
  FPS_HIP(gemm(5, nullptr));
  // The same ADI map as the forward solve (self-adjoint for symmetric
  // shifts), batched; Gbar lands in each problem's G region (FP64 batch).
  if ((s = run_adi_batch(bt, 0, w, st)) != FPS_OK) return s;
  FPS_HIP(finalize_all(bt, w, 0, 0, st));
  // Fbar of every problem: the output-map GEMMs (two table launches).
  FPS_HIP(gemm(6, (char *)Fbar));
  FPS_HIP(gemm(7, (char *)Fbar));
  return FPS_OK;
}

void fps_batch_destroy(fps_batch *bt) {
  if (!valid_batch(bt)) return;
  bt->magic = 0;
  delete bt;
}

}  // extern "C"
