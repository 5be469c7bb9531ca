// gfx950 FP64 MFMA GEMM for the dense coefficient maps of the spectral
// Poisson solver (Chebyshev <-> C~^(3/2) maps of Sec. 3.4 and Table 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "kernels.hpp"

namespace fps {

namespace {

// ---------------------------------------------------------------------------
// FP64 GEMM on v_mfma_f64_16x16x4f64: C = A B with A row-major (k
// contiguous, lda), B row-major (n contiguous, ldb), C(i, j) at
// C[i*ldci + j*ldcj].  Tile 128 x 128 x 16, four wavefronts in a 2 x 2
// grid, each computing a 64 x 64 quarter as 4 x 4 MFMA blocks; the next
// k-tile is fetched into registers while the current one is multiplied, and
// stashed into the second of two LDS stages.
// Operand layout of the 16x16x4 f64 instruction: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r of lane l
// holds C[4r + l / 16][l % 16].
// Requirements (checked by the launcher): K, lda, ldb multiples of 16 bytes'
// worth of doubles (even) and A, B 16-byte aligned; rows/columns of A and B
// beyond M, N, K must be readable up to the next multiple of the tile (the
// plan pads every operand to multiples of 64 with zeros) -- loads are
// clamped to M and N and zero-filled, so only K needs padding.
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

// order: tile dispatch order of a triangular batch, longest k-range first
// (0: natural; 1 / 2: column tile slowest, ascending / descending; 3 / 4:
// row tile slowest, ascending / descending).  Workgroups start in id order,
// so the short tiles fill the tail instead of the long ones.
struct GemmBatch {
  GemmProb p[4];
  int order;
};

constexpr int GBM = 128, GBN = 128, GBK = 16, GPAD = 2;
static_assert(GBM == kGemmTile && GBN == kGemmTile, "tile size shared with the edge split");

// k-range [klo, khi) of tile (bx, by) after the triangular skips.
__host__ __device__ inline void tile_krange(const GemmProb &g, int bx, int by, int64_t *klo_out,
                                            int64_t *khi_out) {
  const int64_t i0 = (int64_t)by * GBM, j0 = (int64_t)bx * GBN;
  int64_t klo = 0;
  if (g.triA) klo = i0 + g.offA > klo ? i0 + g.offA : klo;
  if (g.triB) klo = j0 + g.offB > klo ? j0 + g.offB : klo;
  klo = klo / GBK * GBK;
  int64_t khi = g.K;
  if (g.triAu) {
    const int64_t e = i0 + GBM - 1 + g.offAu + 1;
    khi = e < khi ? e : khi;
  }
  if (g.triBu) {
    const int64_t e = j0 + GBN - 1 + g.offBu + 1;
    khi = e < khi ? e : khi;
  }
  khi = (khi + GBK - 1) / GBK * GBK;
  if (khi > g.K) khi = g.K;
  *klo_out = klo;
  *khi_out = khi;
}

// One 128 x 128 output tile (column tile bx, row tile by) of problem g.
// Two LDS stages (As, Bs and As2, Bs2): the next k-tile is stashed into the
// stage not being read, so one barrier per k-tile suffices (68 KB of LDS, two
// workgroups per compute unit).
__device__ __forceinline__ void gemm_tile(const GemmProb &g, const int bx, const int by,
                                          double (*As)[GBK + 1], double (*Bs)[GBN + GPAD],
                                          double (*As2)[GBK + 1], double (*Bs2)[GBN + GPAD]) {
  const int64_t i0 = (int64_t)by * GBM, j0 = (int64_t)bx * GBN;
  if (i0 >= g.M || j0 >= g.N) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wy = wid >> 1, wx = wid & 1;
  int64_t klo, khi;
  tile_krange(g, bx, by, &klo, &khi);

  // Loader mapping.  A tile 128 x 16: thread t reads row t/2, k-run (t%2)*8..+8.
  // B tile 16 x 128: thread t reads k-row t/16, the column pairs bc + 32 q
  // (bc = 2 (t%16), q = 0..3), so the 16 threads of a row read and stash
  // 256 contiguous bytes per q (no LDS bank conflicts on the stash).
  const int ar = tid >> 1, ak = (tid & 1) * 8;
  const int bk = tid >> 4, bc = (tid & 15) * 2;
  const int64_t arow = i0 + ar < g.M ? i0 + ar : g.M - 1;
  const double az = i0 + ar < g.M ? 1.0 : 0.0;
  const double *__restrict__ Ap = g.A + arow * g.sai + ak;
  const double *__restrict__ Bp = g.B + (int64_t)bk * g.sbk + j0 + bc;
  const bool bfull = j0 + bc + 3 * 32 + 2 <= g.N;

  dbl2 ra[4], rb[4];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) ra[q] = *(const dbl2 *)(Ap + k0 + 2 * q);
    const double *bp = Bp + k0 * g.sbk;
    if (bfull) {
#pragma unroll
      for (int q = 0; q < 4; ++q) rb[q] = *(const dbl2 *)(bp + 32 * q);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t jj = j0 + bc + 32 * q;
        rb[q].x = jj < g.N ? bp[32 * q] : 0.0;
        rb[q].y = jj + 1 < g.N ? bp[32 * q + 1] : 0.0;
      }
    }
  };
  // A is kept row-major in LDS ([row][k], one double of padding): the
  // stash writes each thread's k-run in place and the fragment reads
  // (16 rows at one k per quarter-wave) hit distinct banks.
  auto stash_to = [&](double (*Ad)[GBK + 1], double (*Bd)[GBN + GPAD]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Ad[ar][ak + 2 * q] = az * ra[q].x;
      Ad[ar][ak + 2 * q + 1] = az * ra[q].y;
      *(dbl2 *)&Bd[bk][bc + 32 * q] = rb[q];
    }
  };


  dbl4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  // 16 x 16 blocks of this wavefront's 64 x 64 quarter that hold output
  // entries: a thin last tile (a few rows or columns past whole tiles) skips
  // the products of its empty blocks (uniform per wavefront).
  const int64_t mrem = g.M - (i0 + wy * 64), nrem = g.N - (j0 + wx * 64);
  const int na = mrem >= 64 ? 4 : mrem <= 0 ? 0 : (int)((mrem + 15) / 16);
  const int nb = nrem >= 64 ? 4 : nrem <= 0 ? 0 : (int)((nrem + 15) / 16);
  const bool full = na == 4 && nb == 4;
  // the products of one k-tile from the stage (Ar, Br)
  auto mma = [&](double (*Ar)[GBK + 1], double (*Br)[GBN + GPAD]) {
#pragma unroll
    for (int ks = 0; ks < GBK; ks += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = Ar[wy * 64 + a * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Br[ks + (lane >> 4)][wx * 64 + b * 16 + (lane & 15)];
      if (full) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      } else {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (a < na && b < nb)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
  };
  if (klo < khi) {
    fetch(klo);
    stash_to(As, Bs);
    __syncthreads();
    // stage s is read in k-tile t while stage 1 - s receives tile t + 1; the
    // barrier after the stash orders both the stash before the next tile's
    // reads and this tile's reads before the stash that follows
    int t = 0;
    for (int64_t k0 = klo; k0 < khi; k0 += GBK, ++t) {
      const bool more = k0 + GBK < khi;
      if (more) fetch(k0 + GBK);
      const bool odd = (t & 1) != 0;
      mma(odd ? As2 : As, odd ? Bs2 : Bs);
      if (more) stash_to(odd ? As : As2, odd ? Bs : Bs2);
      __syncthreads();
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + wy * 64 + a * 16 + 4 * r + (lane >> 4);
        const int64_t gj = j0 + wx * 64 + b * 16 + (lane & 15);
        if (gi < g.M && gj < g.N) g.C[gi * g.sci + gj * g.scj] = acc[a][b][r];
      }
}

__global__ __launch_bounds__(256, 2) void k_gemm(GemmBatch batch) {
  __shared__ double As[GBM][GBK + 1], As2[GBM][GBK + 1];
  __shared__ double Bs[GBK][GBN + GPAD], Bs2[GBK][GBN + GPAD];
  int bx = blockIdx.x, by = blockIdx.y, z = blockIdx.z;
  if (batch.order != 0) {
    const int nt = gridDim.x, mt = gridDim.y, nz = gridDim.z;
    const int L = blockIdx.x + nt * (blockIdx.y + mt * blockIdx.z);
    if (batch.order <= 2) {
      const int c = L / (mt * nz), rem = L % (mt * nz);
      bx = batch.order == 1 ? c : nt - 1 - c;
      z = rem / mt;
      by = rem % mt;
    } else {
      const int r = L / (nt * nz), rem = L % (nt * nz);
      by = batch.order == 3 ? r : mt - 1 - r;
      z = rem / nt;
      bx = rem % nt;
    }
  }
  gemm_tile(batch.p[z], bx, by, As, Bs, As2, Bs2);
}

// Table-driven GEMM: workgroup g computes tile (local % ntx, local / ntx),
// local = tile_map[2g + 1], of problem tile_map[2g]; operand pointers are
// rebased per GemmDesc base ids.
__device__ __forceinline__ const double *rebase(const double *p, int id, char *ws, char *out) {
  return id == 1 ? (const double *)(ws + (intptr_t)p)
                 : id == 2 ? (const double *)(out + (intptr_t)p) : p;
}

__global__ __launch_bounds__(256, 2) void k_gemm_table(const GemmDesc *__restrict__ d,
                                                       const int *__restrict__ tile_map, char *ws,
                                                       char *out) {
  __shared__ double As[GBM][GBK + 1], As2[GBM][GBK + 1];
  __shared__ double Bs[GBK][GBN + GPAD], Bs2[GBK][GBN + GPAD];
  const int k = __builtin_amdgcn_readfirstlane(tile_map[2 * blockIdx.x]);
  const int local = __builtin_amdgcn_readfirstlane(tile_map[2 * blockIdx.x + 1]);
  const GemmDesc &e = d[k];
  GemmProb g = e.p;
  g.A = rebase(g.A, e.abase, ws, out);
  g.B = rebase(g.B, e.bbase, ws, out);
  g.C = (double *)rebase(g.C, e.cbase, ws, out);
  gemm_tile(g, local % e.ntx, local / e.ntx, As, Bs, As2, Bs2);
}

// Columns tn.. of every row of a table problem: one wavefront per row,
// lanes striding over k with coalesced loads of the row, then a butterfly
// sum across the wavefront (fixed order, so the result is reproducible).
// kRows rows per wavefront iteration keep their loads in flight together;
// rows with k contiguous, even K and a 16-byte aligned start are read two
// k at a time (kVecRows rows in flight).  Workgroup b serves problem
// b % nprob, so problems that read different parts of the same rows (the
// parity blocks of one array) read them at the same time.
__global__ __launch_bounds__(256) void k_gemm_edge_cols(const GemmDesc *__restrict__ d, int nprob,
                                                        int64_t tn, char *ws, char *out) {
  constexpr int kRows = 4, kVecRows = 8;
  const GemmDesc &e = d[blockIdx.x % nprob];
  const double *__restrict__ A = rebase(e.p.A, e.abase, ws, out);
  const double *__restrict__ B = rebase(e.p.B, e.bbase, ws, out);
  double *__restrict__ C = (double *)rebase(e.p.C, e.cbase, ws, out);
  const int64_t M = e.p.M, N = e.p.N, K = e.p.K;
  const int64_t nn = N < tn ? N : tn;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)(blockIdx.x / nprob) * 4 + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)(gridDim.x / nprob) * 4;
  if (e.p.sak == 1 && !(e.p.sai & 1) && !(K & 1) && !((uintptr_t)A & 15)) {
    for (int64_t i0 = wave * kVecRows; i0 < M; i0 += nwaves * kVecRows) {
      for (int64_t j = nn; j < N; ++j) {
        double acc[kVecRows];
#pragma unroll
        for (int r = 0; r < kVecRows; ++r) acc[r] = 0.0;
        for (int64_t k = 2 * lane; k < K; k += 128) {
          const double b0 = B[k * e.p.sbk + j * e.p.sbj], b1 = B[(k + 1) * e.p.sbk + j * e.p.sbj];
          dbl2 a[kVecRows];
#pragma unroll
          for (int r = 0; r < kVecRows; ++r) {
            const int64_t i = i0 + r < M ? i0 + r : M - 1;
            a[r] = *(const dbl2 *)(A + i * e.p.sai + k);
          }
#pragma unroll
          for (int r = 0; r < kVecRows; ++r) acc[r] = fma(a[r].y, b1, fma(a[r].x, b0, acc[r]));
        }
#pragma unroll
        for (int r = 0; r < kVecRows; ++r) {
          double v = acc[r];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
          if (lane == 0 && i0 + r < M) C[(i0 + r) * e.p.sci + j * e.p.scj] = v;
        }
      }
    }
    return;
  }
  for (int64_t i0 = wave * kRows; i0 < M; i0 += nwaves * kRows) {
    for (int64_t j = nn; j < N; ++j) {
      double acc[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) acc[r] = 0.0;
      for (int64_t k = lane; k < K; k += 64) {
        const double b = B[k * e.p.sbk + j * e.p.sbj];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const int64_t i = i0 + r < M ? i0 + r : M - 1;
          acc[r] = fma(A[i * e.p.sai + k * e.p.sak], b, acc[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        double v = acc[r];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0 && i0 + r < M) C[(i0 + r) * e.p.sci + j * e.p.scj] = v;
      }
    }
  }
}

}  // namespace

hipError_t launch_gemm_edge_cols(const GemmDesc *d, int nprob, int64_t tn, int nblk, char *ws,
                                 char *out, hipStream_t st) {
  if (nprob <= 0 || nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_edge_cols, dim3((unsigned)(nblk * nprob)), dim3(256), 0, st, d, nprob,
                     tn, ws, out);
  return hipGetLastError();
}

bool gemm_operands_ok(const GemmProb &q) {
  return q.sak == 1 && q.sbj == 1 && q.K % GBK == 0 && !(q.sai & 1) && !(q.sbk & 1) &&
         !((uintptr_t)q.A & 15) && !((uintptr_t)q.B & 15) && q.M >= 1 && q.N >= 1;
}

int gemm_tiles(const GemmProb &q, int *ntx) {
  *ntx = (int)((q.N + GBN - 1) / GBN);
  return *ntx * (int)((q.M + GBM - 1) / GBM);
}

hipError_t launch_gemm_table(const GemmDesc *d, const int *tile_map, int ntiles, char *ws,
                             char *out, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_table, dim3((unsigned)ntiles), dim3(256), 0, st, d, tile_map, ws,
                     out);
  return hipGetLastError();
}

std::vector<int> gemm_table_map(const std::vector<GemmDesc> &tab) {
  // every tile of every problem, longest k-range first (workgroups start in
  // id order, so the short tiles fill the tail); ties keep table order
  struct T {
    int64_t work;
    int prob, local;
  };
  std::vector<T> tiles;
  for (size_t k = 0; k < tab.size(); ++k) {
    int ntx = 0;
    const int nt = gemm_tiles(tab[k].p, &ntx);
    for (int l = 0; l < nt; ++l) {
      int64_t klo, khi;
      tile_krange(tab[k].p, l % ntx, l / ntx, &klo, &khi);
      tiles.push_back(T{khi > klo ? khi - klo : 0, (int)k, l});
    }
  }
  std::stable_sort(tiles.begin(), tiles.end(), [](const T &a, const T &b) { return a.work > b.work; });
  std::vector<int> map;
  map.reserve(2 * tiles.size());
  for (const T &t : tiles) {
    map.push_back(t.prob);
    map.push_back(t.local);
  }
  return map;
}

hipError_t launch_gemm(const GemmProb *probs, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (count > 4) return hipErrorInvalidValue;
  GemmBatch b{};
  int64_t mt = 1, nt = 1;
  for (int i = 0; i < count; ++i) {
    const GemmProb &q = probs[i];
    // contiguous operands, 16-byte aligned, K padded to the k-tile
    if (!gemm_operands_ok(q)) return hipErrorInvalidValue;
    b.p[i] = probs[i];
    mt = probs[i].M > mt * GBM ? (probs[i].M + GBM - 1) / GBM : mt;
    nt = probs[i].N > nt * GBN ? (probs[i].N + GBN - 1) / GBN : nt;
  }
  // Longest-first order when every problem has the same one-sided
  // triangular structure: the k-range of a tile then shrinks along one tile
  // index (triB: klo grows with the column tile, triBu: khi grows with it;
  // triA / triAu likewise with the row tile).
  const GemmProb &f = probs[0];
  bool same = true;
  for (int i = 1; i < count; ++i) {
    const GemmProb &q = probs[i];
    same = same && q.triA == f.triA && q.triB == f.triB && q.triAu == f.triAu &&
           q.triBu == f.triBu;
  }
  const bool rowwise = f.triA || f.triAu, colwise = f.triB || f.triBu;
  if (same && colwise && !rowwise && !(f.triB && f.triBu))
    b.order = f.triB ? 1 : 2;
  else if (same && rowwise && !colwise && !(f.triA && f.triAu))
    b.order = f.triA ? 3 : 4;
  dim3 grid((unsigned)nt, (unsigned)mt, (unsigned)count);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, b);
  return hipGetLastError();
}

}  // namespace fps
