// Small dense FP64 kernels on N_b x N_b matrices (N_b up to a few thousand).
//
//  * potrf: blocked right-looking Cholesky S = L L^T (Sec. 3.4 Alg. 3 step 2;
//    the paper uses ScaLAPACK pXpotrf).  32x32 diagonal blocks are factored
//    in LDS by one work-group, which also inverts them for the panel solve.
//  * trtri_t: W = L^-T (Alg. 3 step 3; the paper uses pXtrtri), block row by
//    block row from the diagonal-block inverses.
//  * jacobi: symmetric eigensolver for the projected Hamiltonian (Sec. 3.5
//    step ii).  Cyclic Jacobi in round-robin (parallel) order: each round
//    rotates n/2 disjoint (p,q) planes at once; the 2x2 block of every pair
//    of planes is updated by one thread from the previous round's matrix
//    (double buffered), so a round is one launch with no atomics.  Many
//    independent eigenproblems share each round's launch (the batched
//    workload's projected Hamiltonians), with one convergence check per
//    sweep for all of them.
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

// One problem of a batched Jacobi round: matrices A (n x n) and V, each
// double buffered (A[b] / V[b]), the buffer holding the matrix at the start
// of the sweep (par0), and the range of blocks of the round launch that
// update it.
struct JacProb {
  double *A[2], *V[2];
  int n, np, par0;
  int64_t first_block, nblocks;
};

// Round r of a sweep for every problem in the table.  Each problem does
// exactly one sweep (rounds 0 .. np-2) per batched sweep and idles in later
// rounds, so its sequence of operations is the one of a solve on its own.
__global__ __launch_bounds__(256) void jacobi_round_kernel(const JacProb *__restrict__ probs, int nprob, int r) {
  // problem of this block: last entry with first_block <= blockIdx.x
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (probs[mid].first_block <= (int64_t)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const JacProb &J = probs[lo];
  const int n = J.n, np = J.np, P = np / 2;
  if (r >= np - 1) return;                       // this problem's sweep is complete
  const int par = (J.par0 + r) & 1;
  const double *__restrict__ A = J.A[par];
  double *__restrict__ An = J.A[par ^ 1];
  const double *__restrict__ V = J.V[par];
  double *__restrict__ Vn = J.V[par ^ 1];
  const int64_t nA = (int64_t)P * P;
  const int64_t total = nA + (int64_t)n * P;
  const int64_t t = ((int64_t)blockIdx.x - J.first_block) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  if (t < nA) {
    const int I = (int)(t / P), Jc = (int)(t % P);
    const int pI = rr_index(I, r, np), qI = rr_index(np - 1 - I, r, np);
    const int pJ = rr_index(Jc, r, np), qJ = rr_index(np - 1 - Jc, r, np);
    double cI, sI, tI, cJ, sJ, tJ;
    jrot(A, n, pI, qI, cI, sI, tI);
    jrot(A, n, pJ, qJ, cJ, sJ, tJ);
    if (I == Jc) {
      if (pI >= n || qI >= n) {
        if (pI < n) An[(int64_t)pI * n + pI] = A[(int64_t)pI * n + pI];
        if (qI < n) An[(int64_t)qI * n + qI] = A[(int64_t)qI * n + qI];
        return;
      }
      const double apq = A[(int64_t)pI * n + qI];
      An[(int64_t)pI * n + pI] = A[(int64_t)pI * n + pI] - tI * apq;
      An[(int64_t)qI * n + qI] = A[(int64_t)qI * n + qI] + tI * apq;
      An[(int64_t)pI * n + qI] = 0.0;
      An[(int64_t)qI * n + pI] = 0.0;
      return;
    }
    const bool pIo = pI < n, qIo = qI < n, pJo = pJ < n, qJo = qJ < n;
    const double b00 = (pIo && pJo) ? A[(int64_t)pI * n + pJ] : 0.0;
    const double b01 = (pIo && qJo) ? A[(int64_t)pI * n + qJ] : 0.0;
    const double b10 = (qIo && pJo) ? A[(int64_t)qI * n + pJ] : 0.0;
    const double b11 = (qIo && qJo) ? A[(int64_t)qI * n + qJ] : 0.0;
    // rows: R_I^T B
    const double r00 = cI * b00 - sI * b10, r01 = cI * b01 - sI * b11;
    const double r10 = sI * b00 + cI * b10, r11 = sI * b01 + cI * b11;
    // columns: (R_I^T B) R_J
    if (pIo && pJo) An[(int64_t)pI * n + pJ] = cJ * r00 - sJ * r01;
    if (pIo && qJo) An[(int64_t)pI * n + qJ] = sJ * r00 + cJ * r01;
    if (qIo && pJo) An[(int64_t)qI * n + pJ] = cJ * r10 - sJ * r11;
    if (qIo && qJo) An[(int64_t)qI * n + qJ] = sJ * r10 + cJ * r11;
  } else {
    const int64_t u = t - nA;
    const int row = (int)(u / P), I = (int)(u % P);
    const int pI = rr_index(I, r, np), qI = rr_index(np - 1 - I, r, np);
    double c, s, tt;
    jrot(A, n, pI, qI, c, s, tt);
    const double vp = pI < n ? V[(int64_t)row * n + pI] : 0.0;
    const double vq = qI < n ? V[(int64_t)row * n + qI] : 0.0;
    if (pI < n) Vn[(int64_t)row * n + pI] = c * vp - s * vq;
    if (qI < n) Vn[(int64_t)row * n + qI] = s * vp + c * vq;
  }
}

// out[2k] = sum of squares off the diagonal of problem k's current matrix,
// out[2k+1] = on the diagonal (one work-group per problem)
__global__ __launch_bounds__(1024) void offnorm_kernel(const JacProb *__restrict__ probs, double *__restrict__ out) {
  __shared__ double so[1024], sd[1024];
  const JacProb &J = probs[blockIdx.x];
  const double *A = J.A[J.par0];
  const int n = J.n;
  double o = 0, d = 0;
  const int64_t total = (int64_t)n * n;
  for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int i = (int)(idx / n), jj = (int)(idx % n);
    const double v = A[idx];
    if (i == jj) d += v * v;
    else o += v * v;
  }
  so[threadIdx.x] = o;
  sd[threadIdx.x] = d;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
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

size_t jacobi_work_elems(int n) { return (size_t)3 * n * n + 16; }
size_t jacobi_table_bytes(int njobs) { return (size_t)(njobs > 0 ? njobs : 1) * sizeof(JacProb); }

int jacobi_eigh_batch(const JacobiJob *jobs, int njobs, double tol, int max_sweeps, void *table, double *norms,
                      double *host_norms, hipStream_t s, int *sweeps_done) {
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
    J.V[0] = jb.work + (size_t)n * n;
    J.V[1] = jb.work + (size_t)2 * n * n;
    J.n = n;
    J.np = n + (n & 1);
    J.par0 = 0;
    J.first_block = J.nblocks = 0;
    hipLaunchKernelGGL(eye_kernel, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, J.V[0], n);
    if (n <= 1) active[k] = 0;
  }
  JacProb *dtab = static_cast<JacProb *>(table);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    // convergence of every active problem, one host synchronisation
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
    hipLaunchKernelGGL(offnorm_kernel, dim3((unsigned)act.size()), dim3(1024), 0, s, dtab, norms);
    if (hipMemcpyAsync(host_norms, norms, 2 * act.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
      return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    std::vector<JacProb> run;
    int rmax = 0;
    int64_t blocks = 0;
    for (size_t a = 0; a < act.size(); ++a) {
      const int k = ids[a];
      const double off = host_norms[2 * a], tot = host_norms[2 * a] + host_norms[2 * a + 1];
      bool done = off <= tol * tol * tot;
      if (prev_off[k] >= 0 && off >= prev_off[k] && off <= 1e-20 * tot) done = true;  // stagnated at rounding
      prev_off[k] = off;
      if (done) {
        active[k] = 0;
        continue;
      }
      JacProb &J = all[k];
      const int P = J.np / 2;
      J.first_block = blocks;
      J.nblocks = ((int64_t)P * P + (int64_t)J.n * P + 255) / 256;
      blocks += J.nblocks;
      rmax = std::max(rmax, J.np - 1);
      run.push_back(J);
      J.par0 ^= (J.np - 1) & 1;                   // buffer holding the matrix after this sweep
    }
    if (run.empty()) break;
    if (hipMemcpyAsync(dtab, run.data(), run.size() * sizeof(JacProb), hipMemcpyHostToDevice, s) != hipSuccess)
      return -1;
    for (int r = 0; r < rmax; ++r)
      hipLaunchKernelGGL(jacobi_round_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dtab, (int)run.size(), r);
    // the table is rewritten next sweep: this sweep's launches must have read it
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
  }
  for (int k = 0; k < njobs; ++k) {
    const JacProb &J = all[k];
    hipLaunchKernelGGL(jacobi_sort_kernel, dim3((J.n + 255) / 256), dim3(256), 0, s, J.A[J.par0], J.V[J.par0], J.n,
                       jobs[k].evals, jobs[k].Q);
  }
  if (sweeps_done) *sweeps_done = sweep;
  return 0;
}

int jacobi_eigh(double *A, int n, double *work, double *evals, double *Q, double tol, int max_sweeps,
                double *host_scratch, hipStream_t s, int *sweeps_done) {
  // one problem through the batched driver: the table (one entry) and the two
  // norms live at the end of the work array
  static_assert(sizeof(JacProb) <= 8 * sizeof(double), "one table entry fits the work tail");
  const JacobiJob job{A, n, work, evals, Q};
  double *tail = work + (size_t)3 * n * n;
  return jacobi_eigh_batch(&job, 1, tol, max_sweeps, tail, tail + 8, host_scratch, s, sweeps_done);
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
