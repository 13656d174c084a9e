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
// In-place right multiplication by row panels.
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void rmul_kernel(double *__restrict__ X, int64_t ld, int64_t nrows, int n,
                                                   const double *__restrict__ W, int upper, int mixed, int ldsn) {
  extern __shared__ double panel[];  // R x ldsn
  const int64_t row0 = (int64_t)blockIdx.x * R;
  for (int idx = threadIdx.x; idx < R * n; idx += blockDim.x) {
    int r = idx / n, c = idx - r * n;
    int64_t row = row0 + r;
    panel[r * ldsn + c] = row < nrows ? X[row * ld + c] : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 15, kq = lane >> 4;
  const int ncb = (n + 15) / 16;
  constexpr int RB = R / 16;
  for (int cb = wave; cb < ncb; cb += 4) {
    const int col = cb * 16 + j;
    const bool cok = col < n;
    const int kend = upper ? (((cb + 1) * 16 < n) ? (cb + 1) * 16 : n) : n;
    // mixed: k in [kd, kend) is the 64x64 diagonal block of this column block
    const int kd = mixed ? (cb * 16 / 64) * 64 : 0;
    v4d acc[RB];
    v4f acc32[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      acc[r] = v4d{0, 0, 0, 0};
      acc32[r] = v4f{0, 0, 0, 0};
    }
    for (int k = 0; k < kd; k += 4) {  // FP32 part (mixed only)
      const int kk = k + kq;
      float b = (kk < kend && cok) ? (float)W[(int64_t)kk * n + col] : 0.f;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        float a = kk < n ? (float)panel[(r * 16 + j) * ldsn + kk] : 0.f;
        acc32[r] = mfma16x4(a, b, acc32[r]);
      }
    }
    for (int k = kd; k < kend; k += 4) {  // FP64 part
      const int kk = k + kq;
      double b = (kk < kend && cok) ? W[(int64_t)kk * n + col] : 0.0;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        double a = kk < n ? panel[(r * 16 + j) * ldsn + kk] : 0.0;
        acc[r] = mfma16x4(a, b, acc[r]);
      }
    }
    if (mixed && kd > 0) {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        v4d t = f32acc_to_f64_layout(acc32[r], lane);
        acc[r] += t;
      }
    }
    if (!cok) continue;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int64_t row = row0 + r * 16 + acc_row<double>(kq, q);
        if (row < nrows) X[row * ld + col] = acc[r][q];
      }
  }
}

int rmul_launch(double *X, int64_t ld, int64_t nrows, int n, const double *W, int upper, int mixed,
                hipStream_t s) {
  if (mixed && !upper) return -1;
  const int ldsn = (n % 2 == 0) ? n + 1 : n;
  const size_t lds32 = (size_t)32 * ldsn * sizeof(double);
  const size_t lds16 = (size_t)16 * ldsn * sizeof(double);
  const size_t cap = 160 * 1024;
  if (lds32 <= cap) {
    unsigned grid = (unsigned)((nrows + 31) / 32);
    if (grid == 0) return 0;
    hipLaunchKernelGGL((rmul_kernel<32>), dim3(grid), dim3(256), lds32, s, X, ld, nrows, n, W, upper, mixed, ldsn);
  } else if (lds16 <= cap) {
    unsigned grid = (unsigned)((nrows + 15) / 16);
    if (grid == 0) return 0;
    hipLaunchKernelGGL((rmul_kernel<16>), dim3(grid), dim3(256), lds16, s, X, ld, nrows, n, W, upper, mixed, ldsn);
  } else {
    return -1;
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
