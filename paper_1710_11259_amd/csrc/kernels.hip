// gfx950 kernels of the spectral Poisson solver.
//
// Sweep design (one launch per ADI half-sweep of Algorithm 2):
//   * every lane owns one chain (storage column) and kSeg consecutive
//     positions of it; kWaves wavefronts stacked along the chain form a chunk;
//   * the Thomas recurrences y_k = r_k - l_k y_{k-1} and
//     x_k = ib_k y_k - u_k x_{k+1} use factors of the whole chain (computed
//     once per shift on the host), so splitting a chain only re-associates
//     the recurrences: each piece runs with zero carries and the true carry
//     enters through precomputed multiplier products;
//   * carries between the segments of a chunk go through LDS; carries
//     between chunks are left in a small array, resolved by k_reduce, and
//     folded into the next pass when it reads its input;
//   * the multiply by (A~ - p' I) that Algorithm 2 applies after each solve
//     along the same direction is r - (p + p') x, so no neighbour access is
//     needed; the pass output is stored transposed so that the next pass,
//     which solves along the other direction, again reads whole rows.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fps {

namespace {

template <typename T>
__device__ __forceinline__ double ld_as_double(const T *p) {
  return (double)(*p);
}

template <typename T>
__global__ __launch_bounds__(kCols *kWaves) void k_sweep(SweepArgs a) {
  __shared__ double sh_y[kWaves][kCols];
  __shared__ double sh_x[kWaves][kCols];

  const int lane = threadIdx.x & (kCols - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t npad = a.npad, ms = a.mstride;
  const int64_t col = (int64_t)blockIdx.x * kCols + lane;
  const int by = blockIdx.y;
  const int s = by < a.nc0 ? 0 : 1;
  const int c = by - (s ? a.nc0 : 0);
  const int64_t mps = s ? a.mp1 : a.mp0;
  const int64_t k0 = (int64_t)c * kChunk + (int64_t)w * kSeg;
  const bool active = k0 < mps;
  const int64_t row0 = (s ? a.mp0 : 0) + k0;

  const double *__restrict__ tab = a.tab + (int64_t)s * kNTab * ms;
  const double *__restrict__ tl = tab + T_L * ms + k0;
  const double *__restrict__ tib = tab + T_IB * ms + k0;
  const double *__restrict__ tu = tab + T_U * ms + k0;
  const double *__restrict__ tf1 = tab + T_F1 * ms;
  const double *__restrict__ tbk1 = tab + T_BK1 * ms;

  double y[kSeg];
#pragma unroll
  for (int i = 0; i < kSeg; ++i) y[i] = 0.0;

  if (active) {
    if (a.in != nullptr) {
      const T *__restrict__ in = (const T *)a.in;
      // Producer of `in` solved along this pass's columns: its chain is this
      // storage row, its position is this column.
      const int64_t kap0 = (int64_t)blockIdx.x * kCols;
      const int sp = kap0 >= a.mp0 ? 1 : 0;
      const int64_t kp = col - (sp ? a.mp0 : 0);
      const int64_t cp = (kap0 - (sp ? a.mp0 : 0)) / kChunk;
      const double *tp = a.tab_prev + (int64_t)sp * kNTab * ms;
      const double bf = tp[T_BF2 * ms + kp];
      const double bk = tp[T_BK2 * ms + kp];
      const double *__restrict__ ab = a.ab_prev + ((cp * npad + row0) * 2 + sp) * 2;
#pragma unroll
      for (int i = 0; i < kSeg; ++i) {
        const double v = ld_as_double(in + (row0 + i) * npad + col);
        y[i] = v + ab[i * 4 + 0] * bf + ab[i * 4 + 1] * bk;
      }
    }
    if (a.g != nullptr) {
      const double *__restrict__ g = a.g;
#pragma unroll
      for (int i = 0; i < kSeg; ++i) y[i] += a.sg * g[(row0 + i) * npad + col];
    }
  }

  // Forward elimination with zero carry-in.
  {
    double carry = 0.0;
#pragma unroll
    for (int i = 0; i < kSeg; ++i) {
      y[i] = y[i] - tl[i] * carry;
      carry = y[i];
    }
  }
  sh_y[w][lane] = y[kSeg - 1];
  __syncthreads();
  double cf1 = 0.0;
  for (int v = 0; v < w; ++v) {
    const int64_t last = (int64_t)c * kChunk + (int64_t)v * kSeg + kSeg - 1;
    cf1 = sh_y[v][lane] + tf1[last] * cf1;
  }
#pragma unroll
  for (int i = 0; i < kSeg; ++i) y[i] += tf1[k0 + i] * cf1;
  const double ylast_chunk = y[kSeg - 1];

  // Backward substitution with zero carry-in, fused with the output.
  const double sigma = a.sigma;
  double xnext = 0.0, xfirst = 0.0;
#pragma unroll
  for (int i = kSeg - 1; i >= 0; --i) {
    const double x = y[i] * tib[i] - tu[i] * xnext;
    const double yprev = i > 0 ? y[i - 1] : cf1;
    const double r = y[i] + tl[i] * yprev;  // the input value r_k
    y[i] = a.final_mode ? x : r - sigma * x;
    xnext = x;
    if (i == 0) xfirst = x;
  }
  sh_x[w][lane] = xfirst;
  __syncthreads();
  double cb1 = 0.0;
  for (int v = kWaves - 1; v > w; --v) {
    const int64_t first = (int64_t)c * kChunk + (int64_t)v * kSeg;
    cb1 = sh_x[v][lane] + tbk1[first] * cb1;
  }
  const double coef = (a.final_mode ? 1.0 : -sigma) * cb1;
#pragma unroll
  for (int i = 0; i < kSeg; ++i) y[i] += coef * tbk1[k0 + i];

  // Chunk boundary data for the second-level carries.
  if (w == kWaves - 1) a.lv[(((int64_t)c * 2 + s) * 2 + 0) * npad + col] = ylast_chunk;
  if (w == 0) a.lv[(((int64_t)c * 2 + s) * 2 + 1) * npad + col] = xfirst + tbk1[k0] * cb1;

  if (active) {
    T *__restrict__ out = (T *)a.out;
    if (a.final_mode) {
#pragma unroll
      for (int i = 0; i < kSeg; ++i) out[(row0 + i) * npad + col] = (T)y[i];
    } else {
      T *o = out + col * npad + row0;
#pragma unroll
      for (int i = 0; i < kSeg; ++i) o[i] = (T)y[i];
    }
  }
}

__global__ void k_reduce(const double *__restrict__ lv, const double *__restrict__ ctab,
                         double *__restrict__ ab, double scale, int64_t npad, int nc0, int nc1,
                         int64_t ncmax) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * npad) return;
  const int s = idx >= npad ? 1 : 0;
  const int64_t col = idx - (s ? npad : 0);
  const int nc = s ? nc1 : nc0;
  const double *C = ctab + (int64_t)s * kNCTab * ncmax;
  double cf = 0.0;
  for (int c = 0; c < nc; ++c) {
    ab[(((int64_t)c * npad + col) * 2 + s) * 2 + 0] = cf;
    const double yl = lv[(((int64_t)c * 2 + s) * 2 + 0) * npad + col];
    cf = yl + C[C_F2LAST * ncmax + c] * cf;
  }
  double cb = 0.0;
  for (int c = nc - 1; c >= 0; --c) {
    double *e = ab + (((int64_t)c * npad + col) * 2 + s) * 2;
    const double cfc = e[0];
    e[0] = scale * cfc;
    e[1] = scale * cb;
    const double xf = lv[(((int64_t)c * 2 + s) * 2 + 1) * npad + col];
    cb = xf + C[C_BF2FIRST * ncmax + c] * cfc + C[C_BK2FIRST * ncmax + c] * cb;
  }
}

__global__ void k_finalize(const double *__restrict__ x, const double *__restrict__ ab,
                           const double *__restrict__ tab, double *__restrict__ out, int mode,
                           const double *__restrict__ sinv, int64_t n, int64_t npad, int64_t mp0,
                           int64_t mstride, int64_t ncmax) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (col >= npad) return;
  const int s = r >= mp0 ? 1 : 0;
  const int64_t k = r - (s ? mp0 : 0);
  const int64_t c = k / kChunk;
  const double *tp = tab + (int64_t)s * kNTab * mstride;
  const double *e = ab + ((c * npad + col) * 2 + s) * 2;
  const double v = x[r * npad + col] + e[0] * tp[T_BF2 * mstride + k] + e[1] * tp[T_BK2 * mstride + k];
  if (mode == 0) {
    out[r * npad + col] = v;
    return;
  }
  const int t = col >= mp0 ? 1 : 0;
  const int64_t kc = col - (t ? mp0 : 0);
  const int64_t i = 2 * k + s, j = 2 * kc + t;
  if (i >= n || j >= n) return;
  out[i * n + j] = sinv ? v * sinv[i] * sinv[j] : v;
}

__global__ void k_permute_in(const double *__restrict__ src, double *__restrict__ dst, int64_t n,
                             int64_t npad, int64_t mp0) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (q >= npad) return;
  const int s = r >= mp0 ? 1 : 0, t = q >= mp0 ? 1 : 0;
  const int64_t i = 2 * (r - (s ? mp0 : 0)) + s, j = 2 * (q - (t ? mp0 : 0)) + t;
  dst[r * npad + q] = (i < n && j < n) ? src[i * n + j] : 0.0;
}

__global__ __launch_bounds__(256) void k_transpose(const double *__restrict__ src,
                                                   double *__restrict__ dst, int64_t npad) {
  __shared__ double tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  for (int i = ty; i < 64; i += 4) tile[i][tx] = src[(r0 + i) * npad + c0 + tx];
  __syncthreads();
  for (int i = ty; i < 64; i += 4) dst[(c0 + i) * npad + r0 + tx] = tile[tx][i];
}

__global__ void k_fill(double *__restrict__ dst, int64_t count, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = v;
}

// ---------------------------------------------------------------------------
// FP64 GEMM on v_mfma_f64_16x16x4f64.  Tile 64 x 64 x 16, 4 wavefronts, each
// computing a 32 x 32 quarter as 2 x 2 MFMA blocks.  Operand layout of the
// 16x16x4 f64 instruction: lane l holds A[l%16][l/16] and B[l/16][l%16];
// accumulator register r of lane l is C[4*r + l/16][l%16].
typedef double dbl4 __attribute__((ext_vector_type(4)));

struct GemmBatch {
  GemmProb p[4];
};

constexpr int GBM = 64, GBN = 64, GBK = 16;

__global__ __launch_bounds__(256) void k_gemm(GemmBatch batch) {
  const GemmProb g = batch.p[blockIdx.z];
  const int64_t i0 = (int64_t)blockIdx.y * GBM, j0 = (int64_t)blockIdx.x * GBN;
  if (i0 >= g.M || j0 >= g.N) return;
  __shared__ double As[GBK][GBM + 1];
  __shared__ double Bs[GBK][GBN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wy = wid >> 1, wx = wid & 1;

  int64_t klo = 0;
  if (g.triA) klo = i0 + g.offA > klo ? i0 + g.offA : klo;
  if (g.triB) klo = j0 + g.offB > klo ? j0 + g.offB : klo;
  klo = klo / GBK * GBK;

  dbl4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

  const bool a_kfast = g.sak <= g.sai;
  const bool b_jfast = g.sbj <= g.sbk;
  for (int64_t k0 = klo; k0 < g.K; k0 += GBK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int ii, kk;
      if (a_kfast) {
        kk = e % GBK;
        ii = e / GBK;
      } else {
        ii = e % GBM;
        kk = e / GBM;
      }
      const int64_t gi = i0 + ii, gk = k0 + kk;
      As[kk][ii] = (gi < g.M && gk < g.K) ? g.A[gi * g.sai + gk * g.sak] : 0.0;
      int jj, kb;
      if (b_jfast) {
        jj = e % GBN;
        kb = e / GBN;
      } else {
        kb = e % GBK;
        jj = e / GBK;
      }
      const int64_t gj = j0 + jj, gkb = k0 + kb;
      Bs[kb][jj] = (gj < g.N && gkb < g.K) ? g.B[gkb * g.sbk + gj * g.sbj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GBK; ks += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[ks + (lane >> 4)][wy * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[ks + (lane >> 4)][wx * 32 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + wy * 32 + a * 16 + 4 * r + (lane >> 4);
        const int64_t gj = j0 + wx * 32 + b * 16 + (lane & 15);
        if (gi < g.M && gj < g.N) g.C[gi * g.sci + gj * g.scj] = acc[a][b][r];
      }
}

}  // namespace

template <typename T>
hipError_t launch_sweep(const SweepArgs &a, hipStream_t st) {
  const int nchunks = a.nc0 + a.nc1;
  if (a.npad % kCols != 0 || nchunks <= 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(a.npad / kCols), (unsigned)nchunks);
  hipLaunchKernelGGL(k_sweep<T>, grid, dim3(kCols * kWaves), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_sweep<double>(const SweepArgs &, hipStream_t);
template hipError_t launch_sweep<float>(const SweepArgs &, hipStream_t);

hipError_t launch_reduce(const double *lv, const double *ctab, double *ab, double scale,
                         int64_t npad, int nc0, int nc1, int64_t ncmax, hipStream_t st) {
  const int64_t total = 2 * npad;
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, lv, ctab,
                     ab, scale, npad, nc0, nc1, ncmax);
  return hipGetLastError();
}

hipError_t launch_finalize(const double *x, const double *ab, const double *tab, double *out,
                           int mode, const double *sinv, int64_t n, int64_t npad, int64_t mp0,
                           int64_t mstride, int64_t ncmax, hipStream_t st) {
  dim3 grid((unsigned)((npad + 255) / 256), (unsigned)npad);
  hipLaunchKernelGGL(k_finalize, grid, dim3(256), 0, st, x, ab, tab, out, mode, sinv, n, npad,
                     mp0, mstride, ncmax);
  return hipGetLastError();
}

hipError_t launch_permute_in(const double *src, double *dst, int64_t n, int64_t npad, int64_t mp0,
                             hipStream_t st) {
  dim3 grid((unsigned)((npad + 255) / 256), (unsigned)npad);
  hipLaunchKernelGGL(k_permute_in, grid, dim3(256), 0, st, src, dst, n, npad, mp0);
  return hipGetLastError();
}

hipError_t launch_transpose(const double *src, double *dst, int64_t npad, hipStream_t st) {
  if (npad % 64 != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)(npad / 64), (unsigned)(npad / 64));
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, st, src, dst, npad);
  return hipGetLastError();
}

hipError_t launch_fill(double *dst, int64_t count, double v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, dst, count,
                     v);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmProb *probs, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (count > 4) return hipErrorInvalidValue;
  GemmBatch b{};
  int64_t mt = 1, nt = 1;
  for (int i = 0; i < count; ++i) {
    b.p[i] = probs[i];
    mt = probs[i].M > mt * GBM ? (probs[i].M + GBM - 1) / GBM : mt;
    nt = probs[i].N > nt * GBN ? (probs[i].N + GBN - 1) / GBN : nt;
  }
  dim3 grid((unsigned)nt, (unsigned)mt, (unsigned)count);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, b);
  return hipGetLastError();
}

}  // namespace fps
