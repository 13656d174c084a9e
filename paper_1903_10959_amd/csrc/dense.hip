// Tall-skinny FP64 products of CholGS and Rayleigh-Ritz on MFMA.
//
//  * gram: G = A^T B, lower triangle only (Sec. 3.4 step 1, computing only the
//    lower-triangular part of the Hermitian overlap; Sec. 3.5 the projected
//    Hamiltonian the same way).  Mixed variant (eq. overlapmixedprec): FP64 on
//    the 64x64 diagonal blocks, FP32 inputs/products on the rest.
//  * rmul: X <- X W in place by row panels (Sec. 3.4 step 4, X L^-T; Sec. 3.5
//    subspace rotation X Q).  The paper's outer blocking over rows (B^d) keeps
//    only a panel of the output in extra memory; here a panel of R rows is
//    staged in LDS and overwritten in place.
//  * resid: column norms ||HX_j - lam_j X_j||.
#include "common.hpp"
#include "kernels.hpp"

#include <cmath>

namespace chfsi {

static constexpr int GT = 128;  // gram output tile (4 waves x 64x64)

// lower-triangle tile enumeration t -> (ti, tj), ti >= tj
__device__ __forceinline__ void tri_tile(int t, int &ti, int &tj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

template <typename T>
__device__ __forceinline__ void gram_wave(const double *__restrict__ A, int64_t lda, const double *__restrict__ B,
                                          int64_t ldb, int64_t r0, int64_t r1, int n, int i0, int j0, int lane,
                                          double *__restrict__ out /* 128-wide tile row base at (i0,j0) */) {
  typedef typename acc4<T>::type acc_t;
  const int j = lane & 15, kq = lane >> 4;
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  bool icol[4], jcol[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    icol[a] = i0 + a * 16 + j < n;
    jcol[a] = j0 + a * 16 + j < n;
  }
  for (int64_t k = r0; k < r1; k += 4) {
    const int64_t row = k + kq;
    const bool rok = row < r1;
    T av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      av[a] = (rok && icol[a]) ? (T)A[row * lda + i0 + a * 16 + j] : T(0);
      bv[a] = (rok && jcol[a]) ? (T)B[row * ldb + j0 + a * 16 + j] : T(0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x4(av[a], bv[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int ii = a * 16 + acc_row<T>(kq, q);
        int jj = b * 16 + j;
        out[ii * GT + jj] = (double)acc[a][b][q];
      }
}

__global__ __launch_bounds__(256) void gram_kernel(const double *__restrict__ A, int64_t lda,
                                                   const double *__restrict__ B, int64_t ldb, int64_t nrows, int n,
                                                   int ntiles, int64_t rows_per_split, int mixed,
                                                   double *__restrict__ part) {
  const int split = blockIdx.x / ntiles;
  const int t = blockIdx.x - split * ntiles;
  int ti, tj;
  tri_tile(t, ti, tj);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wi = wave >> 1, wj = wave & 1;
  if (ti == tj && wi < wj) return;  // strictly upper quarter of a diagonal tile: never read
  const int64_t r0 = (int64_t)split * rows_per_split;
  int64_t r1 = r0 + rows_per_split;
  if (r1 > nrows) r1 = nrows;
  const int i0 = ti * GT + wi * 64, j0 = tj * GT + wj * 64;
  double *out = part + ((int64_t)split * ntiles + t) * (GT * GT) + (wi * 64) * GT + wj * 64;
  const bool diag64 = (ti == tj) && (wi == wj);
  if (mixed && !diag64)
    gram_wave<float>(A, lda, B, ldb, r0, r1, n, i0, j0, lane, out);
  else
    gram_wave<double>(A, lda, B, ldb, r0, r1, n, i0, j0, lane, out);
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(const double *__restrict__ part, int nsplit, int ntiles,
                                                          int n, double *__restrict__ G) {
  const int64_t total = (int64_t)n * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(idx / n), jj = (int)(idx - (int64_t)i * n);
    if (jj > i) continue;
    int ti = i / GT, tj = jj / GT;
    int t = ti * (ti + 1) / 2 + tj;
    const double *p = part + (int64_t)t * (GT * GT) + (i - ti * GT) * GT + (jj - tj * GT);
    double s = 0;
    for (int sp = 0; sp < nsplit; ++sp) s += p[(int64_t)sp * ntiles * (GT * GT)];
    G[(int64_t)i * n + jj] = s;
    G[(int64_t)jj * n + i] = s;
  }
}

static int gram_ntiles(int n) {
  int nt = (n + GT - 1) / GT;
  return nt * (nt + 1) / 2;
}

int gram_nsplit(int64_t nrows, int n) {
  int ntiles = gram_ntiles(n);
  int64_t want = (2048 + ntiles - 1) / ntiles;           // about 8 work-groups per CU
  int64_t maxs = (nrows + 255) / 256;                    // at least 256 rows per split
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  return (int)want;
}

size_t gram_part_elems(int64_t nrows, int n) {
  return (size_t)gram_nsplit(nrows, n) * gram_ntiles(n) * GT * GT;
}

void gram_launch(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrows, int n, double *part,
                 double *G, int mixed, hipStream_t s) {
  int ntiles = gram_ntiles(n);
  int nsplit = gram_nsplit(nrows, n);
  int64_t rps = (nrows + nsplit - 1) / nsplit;
  rps = (rps + 15) / 16 * 16;
  hipLaunchKernelGGL(gram_kernel, dim3((unsigned)(nsplit * ntiles)), dim3(256), 0, s, A, lda, B, ldb, nrows, n,
                     ntiles, rps, mixed, part);
  int64_t total = (int64_t)n * n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, part, nsplit, ntiles, n, G);
}

// ---------------------------------------------------------------------------
// Right multiplication X <- X W.  Rows are processed in chunks: an LDS-tiled
// MFMA GEMM writes C = X_chunk W into a scratch chunk, a coalesced copy puts
// it back (the paper's outer blocking over rows, which needs only a chunk of
// extra memory).  Work-group tile 128 x 128 (4 waves x 64 x 64), K staged in
// LDS 16 at a time, double buffered.  upper: W upper triangular, so output
// column tile [n0, n0+128) only needs k < n0 + 128.  mixed (upper only): k in
// the 64-wide diagonal block of a wave's columns in FP64, smaller k in FP32.
// ---------------------------------------------------------------------------
static constexpr int MT = 128, NTL = 128, KC = 16;
static constexpr int ALD = KC + 1;   // padded LDS row of the A tile (odd -> no bank conflicts)

template <bool MIXED>
__global__ __launch_bounds__(256) void rmul_gemm_kernel(const double *__restrict__ X, int64_t ld, int64_t row0,
                                                        int64_t nrows, int n, const double *__restrict__ W,
                                                        int upper, double *__restrict__ C, int64_t ldc) {
  __shared__ double As[2][MT * ALD];
  __shared__ double Ws[2][KC * NTL];
  const int nt = (n + NTL - 1) / NTL;
  const int mt = blockIdx.x / nt;
  const int ntile = blockIdx.x - mt * nt;
  const int64_t r0 = row0 + (int64_t)mt * MT;    // first X row of this tile
  const int n0 = ntile * NTL;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wi = wave >> 1, wj = wave & 1;
  const int j = lane & 15, kq = lane >> 4;
  const int kend = upper ? min(n, n0 + NTL) : n;
  const int c0 = n0 + wj * 64;                   // first column of this wave
  const int kdiag = MIXED ? (c0 / 64) * 64 : 0;  // mixed: k >= kdiag is the FP64 diagonal block

  v4d acc[4][4];
  v4f acc32[MIXED ? 4 : 1][MIXED ? 4 : 1];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  if (MIXED) {
#pragma unroll
    for (int a = 0; a < (MIXED ? 4 : 1); ++a)
#pragma unroll
      for (int b = 0; b < (MIXED ? 4 : 1); ++b) acc32[a][b] = v4f{0, 0, 0, 0};
  }

  auto stage = [&](int buf, int k0) {
    // A tile: 128 rows x 16 columns (each row 128 contiguous bytes)
    for (int idx = tid; idx < MT * KC; idx += 256) {
      const int r = idx / KC, c = idx - r * KC;
      const int64_t row = r0 + r;
      const int k = k0 + c;
      As[buf][r * ALD + c] = (row < row0 + nrows && k < n) ? X[row * ld + k] : 0.0;
    }
    // W tile: 16 rows x 128 columns
    for (int idx = tid; idx < KC * NTL; idx += 256) {
      const int r = idx / NTL, c = idx - r * NTL;
      const int k = k0 + r, col = n0 + c;
      Ws[buf][r * NTL + c] = (k < kend && col < n) ? W[(int64_t)k * n + col] : 0.0;
    }
  };

  const int nk = (kend + KC - 1) / KC;
  if (nk > 0) stage(0, 0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) stage(buf ^ 1, (kc + 1) * KC);
    const int kbase = kc * KC;
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kk = ks + kq;
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[buf][(wi * 64 + a * 16 + j) * ALD + kk];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Ws[buf][kk * NTL + wj * 64 + b * 16 + j];
      if (!MIXED || kbase + ks >= kdiag) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x4(av[a], bv[b], acc[a][b]);
      } else {
#pragma unroll
        for (int a = 0; a < (MIXED ? 4 : 1); ++a)
#pragma unroll
          for (int b = 0; b < (MIXED ? 4 : 1); ++b) acc32[a][b] = mfma16x4((float)av[a], (float)bv[b], acc32[a][b]);
      }
    }
    __syncthreads();
  }
  if (MIXED && kdiag > 0) {
#pragma unroll
    for (int a = 0; a < (MIXED ? 4 : 1); ++a)
#pragma unroll
      for (int b = 0; b < (MIXED ? 4 : 1); ++b) acc[a][b] += f32acc_to_f64_layout(acc32[a][b], lane);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t rr = (int64_t)mt * MT + wi * 64 + a * 16 + acc_row<double>(kq, q);  // chunk-local row
        const int col = c0 + b * 16 + j;
        if (rr < nrows && col < n) C[rr * ldc + col] = acc[a][b][q];
      }
}

__global__ __launch_bounds__(256) void copy_back_kernel(const double *__restrict__ C, int64_t ldc, double *X,
                                                        int64_t ld, int64_t row0, int64_t nrows, int n) {
  const int64_t total = nrows * (int64_t)n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / n;
    const int c = (int)(t - r * n);
    X[(row0 + r) * ld + c] = C[r * ldc + c];
  }
}

int64_t rmul_chunk_rows(int n) {
  // about 256 MiB of scratch, a multiple of the 128-row tile
  int64_t rows = ((int64_t)1 << 25) / (n > 0 ? n : 1);
  rows = rows / MT * MT;
  if (rows < MT) rows = MT;
  return rows;
}

int rmul_launch(double *X, int64_t ld, int64_t nrows, int n, const double *W, int upper, int mixed,
                double *scratch, hipStream_t s) {
  if (mixed && !upper) return -1;
  const int64_t chunk = rmul_chunk_rows(n);
  const int nt = (n + NTL - 1) / NTL;
  for (int64_t r = 0; r < nrows; r += chunk) {
    const int64_t rows = (nrows - r < chunk) ? nrows - r : chunk;
    const int64_t mts = (rows + MT - 1) / MT;
    if (mixed)
      hipLaunchKernelGGL(rmul_gemm_kernel<true>, dim3((unsigned)(mts * nt)), dim3(256), 0, s, X, ld, r, rows, n, W,
                         upper, scratch, (int64_t)n);
    else
      hipLaunchKernelGGL(rmul_gemm_kernel<false>, dim3((unsigned)(mts * nt)), dim3(256), 0, s, X, ld, r, rows, n, W,
                         upper, scratch, (int64_t)n);
    int64_t total = rows * n;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(copy_back_kernel, dim3((unsigned)blocks), dim3(256), 0, s, scratch, (int64_t)n, X, ld, r,
                       rows, n);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Residual column norms
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void resid_part_kernel(const double *__restrict__ X, int64_t ldx,
                                                         const double *__restrict__ HX, int64_t ldh,
                                                         const double *__restrict__ lam, int64_t nrows, int n,
                                                         int64_t rows_per, double *__restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  int64_t r1 = r0 + rows_per;
  if (r1 > nrows) r1 = nrows;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const double l = lam[c];
    double acc = 0;
    for (int64_t r = r0; r < r1; ++r) {
      double d = HX[r * ldh + c] - l * X[r * ldx + c];
      acc += d * d;
    }
    part[(int64_t)blockIdx.x * n + c] = acc;
  }
}

__global__ void resid_reduce_kernel(const double *__restrict__ part, int nchunk, int n, double *__restrict__ out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double s = 0;
  for (int k = 0; k < nchunk; ++k) s += part[(int64_t)k * n + c];
  out[c] = sqrt(s);
}

int resid_nchunk(int64_t nrows) {
  int64_t c = (nrows + 1023) / 1024;
  if (c > 2048) c = 2048;
  if (c < 1) c = 1;
  return (int)c;
}

void resid_launch(const double *X, int64_t ldx, const double *HX, int64_t ldh, const double *lam, int64_t nrows,
                  int n, double *part, double *resid, hipStream_t s) {
  int nchunk = resid_nchunk(nrows);
  int64_t rows_per = (nrows + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(resid_part_kernel, dim3(nchunk), dim3(256), 0, s, X, ldx, HX, ldh, lam, nrows, n, rows_per,
                     part);
  hipLaunchKernelGGL(resid_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, s, part, nchunk, n, resid);
}

}  // namespace chfsi
