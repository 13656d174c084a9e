// Small dense FP64 kernels on N_b x N_b matrices (N_b up to a few thousand).
//
//  * potrf: blocked right-looking Cholesky S = L L^T (Sec. 3.4 Alg. 3 step 2;
//    the paper uses ScaLAPACK pXpotrf).  32x32 diagonal blocks are factored
//    in LDS by one work-group, which also inverts them for the panel solve.
//  * trtri_t: W = L^-T (Alg. 3 step 3; the paper uses pXtrtri), block row by
//    block row from the diagonal-block inverses.
//  * jacobi: symmetric eigensolver for the projected Hamiltonian (Sec. 3.5
//    step ii).  Block-cyclic Jacobi: blocks of 32 indices paired in
//    round-robin (parallel) order; each pair's 64 x 64 submatrix gets a sweep
//    of plane rotations in LDS, and the accumulated 64 x 64 rotations are
//    applied to the whole matrix and to the eigenvectors as small dense
//    products.  Many independent eigenproblems share each launch (the
//    batched workload's projected Hamiltonians), with one convergence check
//    per sweep for all of them.
#include "common.hpp"
#include "kernels.hpp"

#include <cmath>
#include <utility>
#include <vector>

namespace chfsi {

static constexpr int NB = 32;

// Relative pivot below which the overlap counts as numerically singular.
static constexpr double PIVOT_FLOOR = 1e-14;

// Before the factorisation: diag0 = diag(S) (after an optional shift of
// shift_rel * max diag(S) added to the diagonal, the shifted Cholesky remedy).
__global__ __launch_bounds__(1024) void potrf_prep_kernel(double *S, int n, double shift_rel, double *diag0) {
  __shared__ double red[1024];
  double m = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, S[(int64_t)i * n + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double sh = shift_rel * red[0];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double d = S[(int64_t)i * n + i] + sh;
    S[(int64_t)i * n + i] = d;
    diag0[i] = d;
  }
}

// Factor one 32x32 diagonal block in LDS.  Pivot j is accepted when
// d_j > PIVOT_FLOOR * diag0_j; minratio[block] = min_j d_j / diag0_j
// (d_j / S_jj is the squared sine of the angle between column j and the span
// of the columns before it, the loss-of-orthogonality indicator).
__global__ __launch_bounds__(256) void potrf_diag_kernel(double *S, int n, int k0, double *dinv, int *flag,
                                                         const double *diag0, double *minratio) {
  __shared__ double a[NB][NB + 1];
  __shared__ double z[NB][NB + 1];
  const int kw = min(NB, n - k0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
    int i = idx / NB, jj = idx % NB;
    a[i][jj] = (i < kw && jj < kw && jj <= i) ? S[(int64_t)(k0 + i) * n + k0 + jj] : 0.0;
    z[i][jj] = 0.0;
  }
  __syncthreads();
  double rmin = 1.0;
  for (int jj = 0; jj < kw; ++jj) {
    double d = a[jj][jj];
    __syncthreads();
    const double ref = diag0[k0 + jj];
    const double ratio = ref > 0.0 ? d / ref : -1.0;
    rmin = fmin(rmin, ratio);
    double ljj = sqrt(d);
    if (!(ratio > PIVOT_FLOOR) || !(ljj - ljj == 0.0)) {
      if (tid == 0 && *flag == 0) *flag = k0 + jj + 1;
      ljj = __builtin_nan("");
    }
    if (tid == 0) a[jj][jj] = ljj;
    for (int i = jj + 1 + tid; i < kw; i += blockDim.x) a[i][jj] /= ljj;
    __syncthreads();
    const int m = kw - jj - 1;  // trailing size
    for (int idx = tid; idx < m * m; idx += blockDim.x) {
      int i = jj + 1 + idx / m, k = jj + 1 + idx % m;
      if (k <= i) a[i][k] -= a[i][jj] * a[k][jj];
    }
    __syncthreads();
  }
  if (tid == 0) minratio[k0 / NB] = rmin;
  // inverse of the lower-triangular diagonal block, one column per thread
  if (tid < kw) {
    const int c = tid;
    z[c][c] = 1.0 / a[c][c];
    for (int i = c + 1; i < kw; ++i) {
      double s = 0;
      for (int m = c; m < i; ++m) s += a[i][m] * z[m][c];
      z[i][c] = -s / a[i][i];
    }
  }
  __syncthreads();
  double *dz = dinv + (int64_t)(k0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
    int i = idx / NB, jj = idx % NB;
    if (i < kw && jj < kw && jj <= i) S[(int64_t)(k0 + i) * n + k0 + jj] = a[i][jj];
    dz[idx] = (i < kw && jj < kw) ? z[i][jj] : 0.0;
  }
}

// L[i, k0:k0+kw] = S[i, k0:k0+kw] Z^T for rows i >= k0+kw (Z = inverse diagonal block)
__global__ __launch_bounds__(256) void potrf_panel_kernel(double *S, int n, int k0, const double *dinv) {
  __shared__ double z[NB][NB + 1];
  __shared__ double rows[64][NB + 1];
  const int kw = min(NB, n - k0);
  const int r0 = k0 + kw + blockIdx.x * 64;
  const int tid = threadIdx.x;
  const double *dz = dinv + (int64_t)(k0 / NB) * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) z[idx / NB][idx % NB] = dz[idx];
  for (int idx = tid; idx < 64 * NB; idx += blockDim.x) {
    int r = idx / NB, c = idx % NB;
    int i = r0 + r;
    rows[r][c] = (i < n && c < kw) ? S[(int64_t)i * n + k0 + c] : 0.0;
  }
  __syncthreads();
  const int r = tid >> 2;
  const int cbeg = (tid & 3) * 8;
  const int i = r0 + r;
  if (i >= n) return;
  for (int c = cbeg; c < cbeg + 8 && c < kw; ++c) {
    double s = 0;
    for (int t = 0; t <= c; ++t) s += rows[r][t] * z[c][t];
    S[(int64_t)i * n + k0 + c] = s;
  }
}

// S[i][j] -= sum_t L[i][k0+t] L[j][k0+t] on the trailing lower triangle
__global__ __launch_bounds__(256) void potrf_update_kernel(double *S, int n, int k0) {
  __shared__ double li[NB][NB + 1];
  __shared__ double lj[NB][NB + 1];
  const int kw = min(NB, n - k0);
  const int k1 = k0 + kw;
  int t = blockIdx.x;
  int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int i0 = k1 + ti * NB, j0 = k1 + tj * NB;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
    int r = idx / NB, c = idx % NB;
    li[r][c] = (i0 + r < n && c < kw) ? S[(int64_t)(i0 + r) * n + k0 + c] : 0.0;
    lj[r][c] = (j0 + r < n && c < kw) ? S[(int64_t)(j0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
    int r = idx / NB, c = idx % NB;
    int i = i0 + r, jj = j0 + c;
    if (i >= n || jj >= n || jj > i) continue;
    double s = 0;
    for (int q = 0; q < kw; ++q) s += li[r][q] * lj[c][q];
    S[(int64_t)i * n + jj] -= s;
  }
}

void potrf_launch(double *S, int n, double *dinv, int *flag, double *diag0, double *minratio, double shift_rel,
                  hipStream_t s) {
  hipLaunchKernelGGL(potrf_prep_kernel, dim3(1), dim3(1024), 0, s, S, n, shift_rel, diag0);
  for (int k0 = 0; k0 < n; k0 += NB) {
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, S, n, k0, dinv, flag, diag0, minratio);
    const int k1 = k0 + NB;
    if (k1 >= n) break;
    const int rest = n - k1;
    hipLaunchKernelGGL(potrf_panel_kernel, dim3((rest + 63) / 64), dim3(256), 0, s, S, n, k0, dinv);
    const int nt = (rest + NB - 1) / NB;
    hipLaunchKernelGGL(potrf_update_kernel, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, S, n, k0);
  }
}

// ---------------------------------------------------------------------------
// W = L^-T.  Z = L^-1 is lower triangular with Z_ii = dinv_i and, for ib > jb,
// Z_{ib,jb} = -dinv_ib * sum_{kb=jb}^{ib-1} L_{ib,kb} Z_{kb,jb}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void trtri_init_kernel(const double *dinv, int n, double *Z) {
  const int64_t total = (int64_t)n * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(idx / n), jj = (int)(idx % n);
    double v = 0;
    if (i / NB == jj / NB) v = dinv[(int64_t)(i / NB) * NB * NB + (i % NB) * NB + (jj % NB)];
    Z[idx] = v;
  }
}

__global__ __launch_bounds__(256) void trtri_row_kernel(const double *L, const double *dinv, int n, int ib,
                                                        double *Z) {
  __shared__ double lb[NB][NB + 1];
  __shared__ double zb[NB][NB + 1];
  __shared__ double tb[NB][NB + 1];
  const int jb = blockIdx.x;  // < ib
  const int tid = threadIdx.x;
  double acc[4] = {0, 0, 0, 0};
  for (int kb = jb; kb < ib; ++kb) {
    for (int idx = tid; idx < NB * NB; idx += blockDim.x) {
      int r = idx / NB, c = idx % NB;
      int i = ib * NB + r, k = kb * NB + c;
      lb[r][c] = (i < n && k < n) ? L[(int64_t)i * n + k] : 0.0;
      int kk = kb * NB + r, jj = jb * NB + c;
      zb[r][c] = (kk < n && jj < n) ? Z[(int64_t)kk * n + jj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int idx = tid + u * 256;
      int r = idx / NB, c = idx % NB;
      double s = 0;
      for (int q = 0; q < NB; ++q) s += lb[r][q] * zb[q][c];
      acc[u] += s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int idx = tid + u * 256;
    tb[idx / NB][idx % NB] = acc[u];
  }
  const double *di = dinv + (int64_t)ib * NB * NB;
  for (int idx = tid; idx < NB * NB; idx += blockDim.x) lb[idx / NB][idx % NB] = di[idx];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int idx = tid + u * 256;
    int r = idx / NB, c = idx % NB;
    double s = 0;
    for (int q = 0; q < NB; ++q) s += lb[r][q] * tb[q][c];
    int i = ib * NB + r, jj = jb * NB + c;
    if (i < n && jj < n) Z[(int64_t)i * n + jj] = -s;
  }
}

__global__ __launch_bounds__(256) void transpose_kernel(const double *Z, int n, double *W) {
  const int64_t total = (int64_t)n * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(idx / n), jj = (int)(idx % n);
    W[idx] = Z[(int64_t)jj * n + i];
  }
}

static unsigned grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (unsigned)b;
}

void trtri_t_launch(const double *L, const double *dinv, int n, double *Z, double *W, hipStream_t s) {
  const int nb = (n + NB - 1) / NB;
  hipLaunchKernelGGL(trtri_init_kernel, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, dinv, n, Z);
  for (int ib = 1; ib < nb; ++ib)
    hipLaunchKernelGGL(trtri_row_kernel, dim3(ib), dim3(256), 0, s, L, dinv, n, ib, Z);
  hipLaunchKernelGGL(transpose_kernel, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, Z, n, W);
}

// ---------------------------------------------------------------------------
// Jacobi eigensolver
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rr_index(int pos, int r, int np) {
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (np - 1);
}

// Rotation (c, s) that zeroes A_pq: J = [[c, s], [-s, c]] on the (p, q) plane.
__device__ __forceinline__ void jrot(const double *A, int n, int p, int q, double &c, double &s, double &t) {
  c = 1.0;
  s = 0.0;
  t = 0.0;
  if (p >= n || q >= n) return;
  const double apq = A[(int64_t)p * n + q];
  if (fabs(apq) < 1e-300) return;
  const double app = A[(int64_t)p * n + p], aqq = A[(int64_t)q * n + q];
  const double tau = (aqq - app) / (2.0 * apq);
  t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// Block-cyclic Jacobi.  The indices are grouped in blocks of JB = 32; a
// block round pairs the blocks in round-robin order (as the scalar method
// pairs indices), and for every pair (I, J) of blocks
//   1. one work-group takes the 64 x 64 submatrix S = A[I u J, I u J] into
//      LDS and rotates it in parallel rounds of 32 disjoint plane rotations,
//      accumulating them in R (64 x 64, orthogonal);
//   2. A <- R^T A R tile by tile (every pair of pairs: one 64 x 64 triple
//      product), into the other buffer;
//   3. V <- V R in place, panel by panel.
// A sweep is one block round g = 0 that rotates the pairs inside each block
// (31 rounds of 16 pairs in I and 16 in J), then nbp - 1 block rounds g >= 1
// (block pairing g - 1) that rotate only the pairs across I and J (32 rounds
// (t, 32 + (t + ir) mod 32)): every index pair once per sweep, a cyclic
// ordering, in 3 nbp launches instead of n - 1.  (Sweeping all 64 indices in
// every block round re-rotates the pairs inside blocks nbp - 1 times per
// sweep; checked on the host, it needs about as many sweeps for twice the
// inner rounds.)
static constexpr int JB = 32, J2 = 64;
static constexpr int OFFP = 32;   // work-groups per problem in the off-norm

// One problem of a batched block-Jacobi round: A (n x n) double buffered
// (A[b]), V updated in place, R the current round's pair rotations
// (npairs x 64 x 64), the buffer holding A at the start of the sweep (par0),
// and the first work-group of this problem in each of the three launches.
struct JacProb {
  double *A[2], *V, *R;
  int n, nbp, par0;
  int64_t first_inner, first_tile, first_panel;
};

__device__ __forceinline__ int jac_find(const JacProb *__restrict__ probs, int nprob, int which) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t f = which == 0 ? probs[mid].first_inner : which == 1 ? probs[mid].first_tile : probs[mid].first_panel;
    if (f <= (int64_t)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// global index of local index i (0..63) of block pair (I, J); >= n: padding
__device__ __forceinline__ int jac_gidx(int i, int I, int J) { return i < JB ? I * JB + i : J * JB + (i - JB); }

// Local pair t (0..31) of inner round ir: inside the blocks (within) or
// across them.
__device__ __forceinline__ void jac_pair(int t, int ir, bool within, int &p, int &q) {
  if (within) {
    const int h = t >> 4, u = t & 15;                // block half, pair in it
    p = JB * h + rr_index(u, ir, JB);
    q = JB * h + rr_index(JB - 1 - u, ir, JB);
  } else {
    p = t;
    q = JB + (t + ir) % JB;
  }
}

// 1. one sweep of the 64-index pair submatrix in LDS; R out
// g: block round of the sweep (0: pairs inside the blocks, pairing 0;
// g >= 1: pairs across the blocks, pairing g - 1).
__global__ __launch_bounds__(1024) void jacobi_inner_kernel(const JacProb *__restrict__ probs, int nprob, int g) {
  __shared__ double S[J2][J2 + 1];
  __shared__ double Rs[J2][J2 + 1];
  __shared__ double cs[J2 / 2], sn[J2 / 2], tn[J2 / 2];
  const JacProb &P = probs[jac_find(probs, nprob, 0)];
  if (g >= P.nbp) return;                          // this problem's sweep is complete
  const int r = g == 0 ? 0 : g - 1;
  const bool within = g == 0;
  const int k = (int)(blockIdx.x - P.first_inner);
  const int n = P.n;
  const int I = rr_index(k, r, P.nbp), J = rr_index(P.nbp - 1 - k, r, P.nbp);
  const double *A = P.A[(P.par0 + g) & 1];
  const int t = threadIdx.x;
  for (int e = t; e < J2 * J2; e += 1024) {
    const int i = e / J2, j = e % J2;
    const int gi = jac_gidx(i, I, J), gj = jac_gidx(j, I, J);
    S[i][j] = (gi < n && gj < n) ? A[(int64_t)gi * n + gj] : 0.0;
    Rs[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  const int nround = within ? JB - 1 : JB;
  // Across the blocks pair b is (b, JB + (b + ir) % JB): column b of R stays
  // with the threads of pair b, and the second column passes each round to
  // the lane of pair b - 1 in the same 32-lane half.  So R lives in
  // registers there (rows 2 a, 2 a + 1 of both columns), with one lane shift
  // per round; inside the blocks the pairing has no such shape and R stays
  // in LDS.
  const int a = t / (J2 / 2), b = t % (J2 / 2);
  const int src = (t & 32) | ((b + 1) & 31);         // lane holding pair b + 1
  double rP[2], rQ[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    rP[h] = 2 * a + h == b ? 1.0 : 0.0;
    rQ[h] = 2 * a + h == JB + b ? 1.0 : 0.0;
  }
  for (int ir = 0; ir < nround; ++ir) {
    if (t < J2 / 2) {
      int p, q;
      jac_pair(t, ir, within, p, q);
      double c = 1.0, s = 0.0, tt = 0.0;
      const double apq = S[p][q];
      if (fabs(apq) >= 1e-300) {
        const double tau = (S[q][q] - S[p][p]) / (2.0 * apq);
        tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        c = 1.0 / sqrt(1.0 + tt * tt);
        s = tt * c;
      }
      cs[t] = c;
      sn[t] = s;
      tn[t] = tt;
    }
    __syncthreads();
    {
      // 2x2 block (pair a rows, pair b columns), one per thread, in place
      int pa, qa, pb, qb;
      jac_pair(a, ir, within, pa, qa);
      jac_pair(b, ir, within, pb, qb);
      if (a == b) {
        const double apq = S[pa][qa];
        S[pa][pa] -= tn[a] * apq;
        S[qa][qa] += tn[a] * apq;
        S[pa][qa] = 0.0;
        S[qa][pa] = 0.0;
      } else {
        const double ca = cs[a], sa = sn[a], cb = cs[b], sb = sn[b];
        const double b00 = S[pa][pb], b01 = S[pa][qb], b10 = S[qa][pb], b11 = S[qa][qb];
        const double r00 = ca * b00 - sa * b10, r01 = ca * b01 - sa * b11;
        const double r10 = sa * b00 + ca * b10, r11 = sa * b01 + ca * b11;
        S[pa][pb] = cb * r00 - sb * r01;
        S[pa][qb] = sb * r00 + cb * r01;
        S[qa][pb] = cb * r10 - sb * r11;
        S[qa][qb] = sb * r10 + cb * r11;
      }
      // R <- R J: rows 2 per thread, pair b
      if (within) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int row = 2 * a + h;
          const double rp = Rs[row][pb], rq = Rs[row][qb];
          Rs[row][pb] = cs[b] * rp - sn[b] * rq;
          Rs[row][qb] = sn[b] * rp + cs[b] * rq;
        }
      } else {
        const double cb = cs[b], sb = sn[b];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double rp = rP[h], rq = rQ[h];
          rP[h] = cb * rp - sb * rq;
          rQ[h] = sb * rp + cb * rq;
          rQ[h] = __shfl(rQ[h], src, 64);              // next round's second column
        }
      }
    }
    __syncthreads();
  }
  double *Rg = P.R + (int64_t)k * J2 * J2;
  if (within) {
    for (int e = t; e < J2 * J2; e += 1024) Rg[e] = Rs[e / J2][e % J2];
  } else {
    // after the shift of the last round this thread holds column JB + (b + nround) % JB
    const int qcol = JB + (b + nround) % JB;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      Rg[(2 * a + h) * J2 + b] = rP[h];
      Rg[(2 * a + h) * J2 + qcol] = rQ[h];
    }
  }
}

// C = op(X) Y for 64 x 64 LDS operands on FP64 MFMA (16x16x4): wave w of 4
// computes rows 16 w .. 16 w + 15 as four 16 x 16 tiles along the columns;
// c[b][q] is row 16 w + acc_row(kq, q), column 16 b + (lane & 15).
// TRANS: X used transposed.
template <bool TRANS>
__device__ __forceinline__ void jac_mm64(const double (*X)[J2 + 1], const double (*Y)[J2 + 1], v4d (&c)[4], int w,
                                         int lane) {
  const int j = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int b = 0; b < 4; ++b) c[b] = v4d{0, 0, 0, 0};
#pragma unroll 4
  for (int kk = 0; kk < J2; kk += 4) {
    const int k = kk + kq;
    const double a = TRANS ? X[k][16 * w + j] : X[16 * w + j][k];   // A[16 w + j][k]
#pragma unroll
    for (int b = 0; b < 4; ++b) c[b] = mfma16x4(a, Y[k][16 * b + j], c[b]);
  }
}

// 2. A_next[P1 rows, P2 cols] = R_P1^T A[P1, P2] R_P2 for every pair of pairs
//    k1 <= k2, with the mirror tile A_next[P2, P1] its transpose
__global__ __launch_bounds__(256) void jacobi_apply_a_kernel(const JacProb *__restrict__ probs, int nprob, int g) {
  __shared__ double T[J2][J2 + 1], R1[J2][J2 + 1], R2[J2][J2 + 1];
  const JacProb &P = probs[jac_find(probs, nprob, 1)];
  if (g >= P.nbp) return;
  const int r = g == 0 ? 0 : g - 1;
  // A is symmetric, so the tile of pairs (k2, k1) is the transpose of that of
  // (k1, k2): only k1 <= k2 are computed, each written with its mirror
  // (tile = k2 (k2 + 1) / 2 + k1)
  const int tile = (int)(blockIdx.x - P.first_tile);
  int k2 = (int)((sqrtf(8.0f * tile + 1.0f) - 1.0f) * 0.5f);
  while (k2 * (k2 + 1) / 2 > tile) --k2;
  while ((k2 + 1) * (k2 + 2) / 2 <= tile) ++k2;
  const int k1 = tile - k2 * (k2 + 1) / 2;
  const int n = P.n;
  const int I1 = rr_index(k1, r, P.nbp), J1 = rr_index(P.nbp - 1 - k1, r, P.nbp);
  const int I2 = rr_index(k2, r, P.nbp), J2b = rr_index(P.nbp - 1 - k2, r, P.nbp);
  const double *A = P.A[(P.par0 + g) & 1];
  double *An = P.A[(P.par0 + g + 1) & 1];
  const double *Rg1 = P.R + (int64_t)k1 * J2 * J2, *Rg2 = P.R + (int64_t)k2 * J2 * J2;
  const int t = threadIdx.x;
  for (int e = t; e < J2 * J2; e += 256) {
    const int i = e / J2, j = e % J2;
    const int gi = jac_gidx(i, I1, J1), gj = jac_gidx(j, I2, J2b);
    T[i][j] = (gi < n && gj < n) ? A[(int64_t)gi * n + gj] : 0.0;
    R1[i][j] = Rg1[e];
    R2[i][j] = Rg2[e];
  }
  __syncthreads();
  const int wv = t >> 6, lane = t & 63, jl = lane & 15, kq = lane >> 4;
  v4d c[4];
  jac_mm64<false>(T, R2, c, wv, lane);             // U = T R2
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) T[16 * wv + acc_row<double>(kq, q)][16 * b + jl] = c[b][q];
  __syncthreads();
  jac_mm64<true>(R1, T, c, wv, lane);              // C = R1^T U
  __syncthreads();                                  // every wave has read U
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) T[16 * wv + acc_row<double>(kq, q)][16 * b + jl] = c[b][q];
  __syncthreads();
  // C to rows of pair k1 x columns of pair k2, C^T to the mirror tile
  for (int e = t; e < J2 * J2; e += 256) {
    const int i = e / J2, j = e % J2;
    const int gi = jac_gidx(i, I1, J1), gj = jac_gidx(j, I2, J2b);
    if (gi < n && gj < n) An[(int64_t)gi * n + gj] = T[i][j];
    if (k1 != k2) {
      const int hi = jac_gidx(i, I2, J2b), hj = jac_gidx(j, I1, J1);
      if (hi < n && hj < n) An[(int64_t)hi * n + hj] = T[j][i];
    }
  }
}

// 3. V[panel rows, P cols] <- V[panel rows, P cols] R_P, in place
__global__ __launch_bounds__(256) void jacobi_apply_v_kernel(const JacProb *__restrict__ probs, int nprob, int g) {
  __shared__ double T[J2][J2 + 1], Rl[J2][J2 + 1];
  const JacProb &P = probs[jac_find(probs, nprob, 2)];
  if (g >= P.nbp) return;
  const int r = g == 0 ? 0 : g - 1;
  const int np2 = P.nbp / 2;
  const int w = (int)(blockIdx.x - P.first_panel);
  const int panel = w / np2, k = w % np2;
  const int n = P.n;
  const int I = rr_index(k, r, P.nbp), J = rr_index(P.nbp - 1 - k, r, P.nbp);
  const double *Rg = P.R + (int64_t)k * J2 * J2;
  const int t = threadIdx.x;
  const int row0 = panel * J2;
  for (int e = t; e < J2 * J2; e += 256) {
    const int i = e / J2, j = e % J2;
    const int gr = row0 + i, gj = jac_gidx(j, I, J);
    T[i][j] = (gr < n && gj < n) ? P.V[(int64_t)gr * n + gj] : 0.0;
    Rl[i][j] = Rg[e];
  }
  __syncthreads();
  const int wv = t >> 6, lane = t & 63, jl = lane & 15, kq = lane >> 4;
  v4d c[4];
  jac_mm64<false>(T, Rl, c, wv, lane);
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gr = row0 + 16 * wv + acc_row<double>(kq, q), gj = jac_gidx(16 * b + jl, I, J);
      if (gr < n && gj < n) P.V[(int64_t)gr * n + gj] = c[b][q];
    }
}

// Squared off-diagonal and diagonal Frobenius norms of each problem's A, as
// OFFP partial sums per problem (work-group part takes rows part*4 + wave,
// stepping by 4 OFFP); the host adds the partials in a fixed order.
__global__ __launch_bounds__(256) void offnorm_kernel(const JacProb *__restrict__ probs, double *__restrict__ out) {
  __shared__ double so[256], sd[256];
  const int a = blockIdx.x / OFFP, part = blockIdx.x % OFFP;
  const JacProb &J = probs[a];
  const double *A = J.A[J.par0];
  const int n = J.n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double o = 0, d = 0;
  for (int i = part * 4 + wave; i < n; i += OFFP * 4) {
    const double *row = A + (int64_t)i * n;
    for (int j = lane; j < n; j += 64) {
      const double v = row[j];
      if (j == i) d += v * v;
      else o += v * v;
    }
  }
  so[threadIdx.x] = o;
  sd[threadIdx.x] = d;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      sd[threadIdx.x] += sd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = so[0];
    out[2 * blockIdx.x + 1] = sd[0];
  }
}

__global__ __launch_bounds__(256) void eye_kernel(double *V, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    V[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
}

// evals ascending; Q[:, rank(i)] = V[:, i]; ties broken by index
__global__ __launch_bounds__(256) void jacobi_sort_kernel(const double *A, const double *V, int n, double *evals,
                                                          double *Q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = A[(int64_t)i * n + i];
  int rank = 0;
  for (int k = 0; k < n; ++k) {
    double dk = A[(int64_t)k * n + k];
    if (dk < di || (dk == di && k < i)) ++rank;
  }
  evals[rank] = di;
  for (int row = 0; row < n; ++row) Q[(int64_t)row * n + rank] = V[(int64_t)row * n + i];
}

static int jac_nbp(int n) {
  const int nblk = (n + JB - 1) / JB;
  return nblk + (nblk & 1);
}

// work: A's second buffer (n^2), V (n^2), the pair rotations
// (nbp/2 x 64 x 64), a tail for the single-problem table (16 doubles) and
// norms (jacobi_norms_elems(1))
static constexpr int JTAIL = 16 + 2 * OFFP;
size_t jacobi_norms_elems(int njobs) { return (size_t)2 * OFFP * (njobs > 0 ? njobs : 1); }
size_t jacobi_work_elems(int n) {
  return (size_t)2 * n * n + (size_t)(jac_nbp(n) / 2) * J2 * J2 + JTAIL;
}
size_t jacobi_table_bytes(int njobs) { return (size_t)(njobs > 0 ? njobs : 1) * sizeof(JacProb); }

int jacobi_eigh_batch(const JacobiJob *jobs, int njobs, double tol, int max_sweeps, void *table, double *norms,
                      double *host_norms, hipStream_t s, int *sweeps_done, int *converged) {
  if (njobs <= 0) return 0;
  std::vector<JacProb> all(njobs);
  std::vector<int> active(njobs, 1);
  std::vector<double> prev_off(njobs, -1.0);
  for (int k = 0; k < njobs; ++k) {
    const JacobiJob &jb = jobs[k];
    const int n = jb.n;
    JacProb &J = all[k];
    J.A[0] = jb.A;
    J.A[1] = jb.work;
    J.V = jb.work + (size_t)n * n;
    J.R = jb.work + (size_t)2 * n * n;
    J.n = n;
    J.nbp = jac_nbp(n);
    J.par0 = 0;
    J.first_inner = J.first_tile = J.first_panel = 0;
    hipLaunchKernelGGL(eye_kernel, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, J.V, n);
    if (n <= 1) active[k] = 0;
  }
  JacProb *dtab = static_cast<JacProb *>(table);
  int sweep = 0;
  for (;; ++sweep) {
    // convergence of every active problem, one host synchronisation (also
    // after the last allowed sweep, so that its result is judged)
    std::vector<JacProb> act;
    std::vector<int> ids;
    for (int k = 0; k < njobs; ++k)
      if (active[k]) {
        act.push_back(all[k]);
        ids.push_back(k);
      }
    if (act.empty()) break;
    if (hipMemcpyAsync(dtab, act.data(), act.size() * sizeof(JacProb), hipMemcpyHostToDevice, s) != hipSuccess)
      return -1;
    hipLaunchKernelGGL(offnorm_kernel, dim3((unsigned)(act.size() * OFFP)), dim3(256), 0, s, dtab, norms);
    if (hipMemcpyAsync(host_norms, norms, 2 * OFFP * act.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
        hipSuccess)
      return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    std::vector<JacProb> run;
    int rmax = 0;
    int64_t n_inner = 0, n_tile = 0, n_panel = 0;
    for (size_t a = 0; a < act.size(); ++a) {
      const int k = ids[a];
      double off = 0, dg = 0;
      for (int q = 0; q < OFFP; ++q) {
        off += host_norms[2 * (a * OFFP + q)];
        dg += host_norms[2 * (a * OFFP + q) + 1];
      }
      const double tot = off + dg;
      bool done = off <= tol * tol * tot;
      if (prev_off[k] >= 0 && off >= prev_off[k] && off <= 1e-20 * tot) done = true;  // stagnated at rounding
      prev_off[k] = off;
      if (done) {
        active[k] = 0;
        continue;
      }
      if (sweep >= max_sweeps) continue;           // out of sweeps: stays unconverged
      JacProb &J = all[k];
      const int np2 = J.nbp / 2;
      J.first_inner = n_inner;
      J.first_tile = n_tile;
      J.first_panel = n_panel;
      n_inner += np2;
      n_tile += (int64_t)np2 * (np2 + 1) / 2;
      n_panel += (int64_t)((J.n + J2 - 1) / J2) * np2;
      rmax = std::max(rmax, J.nbp);                // block rounds g = 0 .. nbp - 1
      run.push_back(J);
      J.par0 ^= J.nbp & 1;                         // buffer holding A after this sweep (nbp is even)
    }
    if (run.empty()) break;
    if (hipMemcpyAsync(dtab, run.data(), run.size() * sizeof(JacProb), hipMemcpyHostToDevice, s) != hipSuccess)
      return -1;
    const int nr = (int)run.size();
    for (int g = 0; g < rmax; ++g) {
      hipLaunchKernelGGL(jacobi_inner_kernel, dim3((unsigned)n_inner), dim3(1024), 0, s, dtab, nr, g);
      hipLaunchKernelGGL(jacobi_apply_a_kernel, dim3((unsigned)n_tile), dim3(256), 0, s, dtab, nr, g);
      hipLaunchKernelGGL(jacobi_apply_v_kernel, dim3((unsigned)n_panel), dim3(256), 0, s, dtab, nr, g);
    }
    // the table is rewritten next sweep: this sweep's launches must have read it
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
  }
  for (int k = 0; k < njobs; ++k) {
    const JacProb &J = all[k];
    hipLaunchKernelGGL(jacobi_sort_kernel, dim3((J.n + 255) / 256), dim3(256), 0, s, J.A[J.par0], J.V, J.n,
                       jobs[k].evals, jobs[k].Q);
  }
  if (sweeps_done) *sweeps_done = sweep;
  int unconv = 0;
  for (int k = 0; k < njobs; ++k) {
    if (converged) converged[k] = active[k] ? 0 : 1;
    unconv += active[k];
  }
  return unconv;
}

int jacobi_eigh(double *A, int n, double *work, double *evals, double *Q, double tol, int max_sweeps,
                double *host_scratch, hipStream_t s, int *sweeps_done) {
  // one problem through the batched driver: the table (one entry) and the
  // norm partials live in the tail of the work array; host_scratch holds at
  // least jacobi_norms_elems(1) doubles
  static_assert(sizeof(JacProb) <= 16 * sizeof(double), "one table entry fits the work tail");
  const JacobiJob job{A, n, work, evals, Q};
  double *tail = work + jacobi_work_elems(n) - JTAIL;
  return jacobi_eigh_batch(&job, 1, tol, max_sweeps, tail, tail + 16, host_scratch, s, sweeps_done, nullptr);
}

__global__ void fill_kernel(double *X, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    X[i] = v;
}
void fill_launch(double *X, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, X, n, v);
}

__global__ void zero_int_kernel(int *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}
void zero_int_launch(int *p, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

}  // namespace chfsi
