// Electrostatics: the discrete Poisson problem (Sec. 2.4 eq.
// phiTotDiscreteSolve) with homogeneous Dirichlet conditions, solved by the
// Jacobi-preconditioned conjugate-gradient method the paper uses for it
// (Sec. 3.2, matrix-free operator).
//
//   A phi = f,  A = 1/(4 pi) int grad N_i . grad N_j,  f = M rho + point charges.
//
// On the uniform Cartesian GLL mesh the assembled stiffness is the Kronecker
// sum k (+) k (+) k weighted by the diagonal 1D masses:
//   (A x)(I,J,K) = s [ m_J m_K sum_I' k(I,I') x(I',J,K) + m_I m_K sum_J' k(J,J') x(I,J',K)
//                    + m_I m_J sum_K' k(K,K') x(I,J,K') ],   s = 1/(4 pi),
// k the assembled 1D Laplacian stiffness (band half-width p), m the 1D GLL
// mass.  This is the matrix-free operator in its assembled form, applied as a
// blocked stencil that reads x about once from HBM and writes y once (16 bytes
// per DoF).
//
// One CG iteration is three launches: the product fused with the partial
// p.q; r -= alpha q with the partials of r.z and r.r; x += alpha p and the new
// direction p = z + beta p.  The two global sums each iteration needs are
// formed where they are used: every work-group of the update sums the
// product's partials (alpha = r.z / p.q), every work-group of the direction
// pass sums the update's (beta = r.z' / r.z and the stop test r.r <=
// tol^2 f.f), each in the same fixed order, so all work-groups hold the same
// bits.  Work-group 0 keeps the results for later launches: r.z alternates
// between two slots by iteration parity, so no work-group reads the slot its
// own launch writes; the stop count, which every work-group of the same
// launch also reads, can only change from "never" to this iteration's number
// plus one, and both values let iteration it run.  Neither z nor diag(A)^-1
// is stored: diag(A) at a node is a sum of three products of 1D values, so
// both vector passes recompute z = r / diag(A), and an iteration moves eight
// arrays of n_dof values.  The
// iteration that meets the tolerance records its number; launches of later
// iterations return at once, so the host launches iterations in groups and
// reads that number between groups.  (Forming p inside the product, where
// the stencil reads it, saves the direction pass but reads two arrays at
// every halo point: measured 2.3x slower per product.  Summing partials in
// the last work-group of each grid instead, every work-group's device-scope
// release writes back its L2: slower still.)
#include "common.hpp"
#include "ctx.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

namespace chfsi {

static constexpr int PB = 256;              // threads per work-group
static constexpr int PR = 1024;             // threads of the single-work-group reductions
static constexpr int MAXG = 2048;           // element-wise grids: at most this many work-groups (grid-stride)
// scalars: r.z of the last two iterations (slot by parity), r.r, f.f, the
// stop threshold tol^2 f.f, the number of iterations done when the tolerance
// was met (kNever until then), alpha of the last update
enum { S_RZ = 0, S_RR = 2, S_FF, S_STOP, S_STOPAT, S_ALPHA, S_NSCAL };
static constexpr double kNever = 9.0e15;

// Sum over the work-group in a fixed order (butterfly within each wave, then
// the wave sums in wave order), so every work-group that sums the same
// values gets the same bits.
template <int NT = PB>
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += sh[w];
  __syncthreads();
  return s;
}

// y = A x with 2.5D blocking.  Work-group = 4 waves; wave w covers 64
// consecutive I (one lane each) and the RY rows J0 + w RY + [0, RY); the
// work-group marches over KB planes K.  Per plane it stages the plane's
// (64 + 2P) x (4 RY + 2P) halo tile of x in LDS (the x- and y-direction
// neighbours); each lane keeps, per row, its z-window of 2P + 1 values in
// registers.  The lane's x-direction band coefficients sit in registers, the
// wave's y- and z-direction ones are wave-uniform (scalar loads), and the
// y-direction sums of a lane's RY rows share one LDS column read of RY + 2P
// values.  The plane tiles are fetched PD planes ahead.  DOT: part[work-group]
// = its share of x . y.
// Grid: ceil(n/64) ceil(n/(4 RY)) ceil(n/KB) work-groups (1D, XCD-grouped).
constexpr int TX = 64;
template <int P, int RY, int KB, int PD, bool DOT>
__global__ __launch_bounds__(PB) void poisson_stencil_kernel(const double *__restrict__ x, double *__restrict__ y,
                                                             const double *__restrict__ kb,
                                                             const double *__restrict__ m, int n, double s,
                                                             const double *__restrict__ scal, int it,
                                                             double *__restrict__ part) {
  constexpr int BW = 2 * P + 1, TY = 4 * RY, WX = TX + 2 * P, WY = TY + 2 * P;
  constexpr int NTL = (WY * WX + PB - 1) / PB;    // tile values per thread
  __shared__ double sh[PB];
  __shared__ double xs[WY][WX];
  if (DOT && it >= scal[S_STOPAT]) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // XCD-grouped block order: the hardware deals consecutive work-groups to the
  // 8 XCDs in turn; the logical index below is contiguous per XCD, and tiles
  // adjacent in J (which share their halo rows) get consecutive logical
  // indices, so their shared rows are fetched into one L2
  const int g = (int)gridDim.x, b = (int)blockIdx.x;
  const int lid = (b & 7) * (g >> 3) + min(b & 7, g & 7) + (b >> 3);
  const int gx = (n + TX - 1) / TX, gy = (n + TY - 1) / TY;
  const int bx = lid % gx, by = (lid / gx) % gy, bz = lid / (gx * gy);
  const int I0 = bx * TX, J0 = by * TY, K0 = bz * KB;
  const int I = I0 + lane;
  const int64_t n2 = (int64_t)n * n;
  const bool ilive = I < n;
  double kx[BW];
#pragma unroll
  for (int d = 0; d < BW; ++d) kx[d] = ilive ? kb[(int64_t)I * BW + d] : 0.0;
  const double mI = ilive ? m[I] : 0.0;
  // this wave's rows (wave-uniform)
  int Jr[RY];
  bool live[RY];
  double mJ[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    Jr[r] = J0 + w * RY + r;
    live[r] = ilive && Jr[r] < n;
    mJ[r] = Jr[r] < n ? m[Jr[r]] : 0.0;
  }
  // z-windows: x(I, J_r, K - P .. K + P), zero outside the mesh (Dirichlet)
  double win[RY][BW];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int64_t col = (int64_t)I + (int64_t)n * Jr[r];
#pragma unroll
    for (int d = 0; d < BW; ++d) {
      const int k = K0 - P + d - 1;                // shifted in at the first plane
      win[r][d] = (live[r] && k >= 0 && k < n) ? x[col + k * n2] : 0.0;
    }
  }
  // the plane tiles are loaded into registers PD planes ahead, in PD sets
  // used in turn (their latency hides behind PD planes of sums), then stored
  // to LDS
  double treg[PD][NTL];
  double wnext[PD][RY];
  auto load_plane = [&](int K, double(&tr)[NTL], double(&wn)[RY]) {
#pragma unroll
    for (int u = 0; u < NTL; ++u) {
      const int e = threadIdx.x + u * PB;
      const int rr = e / WX, cc = e - rr * WX;
      const int i = I0 - P + cc, j = J0 - P + rr;
      tr[u] = (e < WY * WX && i >= 0 && i < n && j >= 0 && j < n) ? x[(int64_t)i + (int64_t)n * j + K * n2] : 0.0;
    }
    const int k = K + P;
#pragma unroll
    for (int r = 0; r < RY; ++r)
      wn[r] = (live[r] && k < n) ? x[(int64_t)I + (int64_t)n * Jr[r] + k * n2] : 0.0;
  };
  double dot = 0;
  const int K1 = min(K0 + KB, n);
  // plane K from the set (tr, wn), which then receives plane K + PD
  auto plane = [&](int K, double(&tr)[NTL], double(&wn)[RY]) {
    __syncthreads();                               // previous plane's tile consumed
#pragma unroll
    for (int u = 0; u < NTL; ++u) {
      const int e = threadIdx.x + u * PB;
      if (e < WY * WX) xs[e / WX][e % WX] = tr[u];
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
#pragma unroll
      for (int d = 0; d < BW - 1; ++d) win[r][d] = win[r][d + 1];
      win[r][BW - 1] = wn[r];
    }
    __syncthreads();
    if (K + PD < K1) load_plane(K + PD, tr, wn);
    const double *kz = kb + (int64_t)K * BW;
    const double mK = m[K];
    double colv[RY + 2 * P];
#pragma unroll
    for (int i = 0; i < RY + 2 * P; ++i) colv[i] = xs[w * RY + i][lane + P];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (!live[r]) continue;
      const double *ky = kb + (int64_t)Jr[r] * BW;
      double sx = 0, sy = 0, sz = 0;
#pragma unroll
      for (int d = 0; d < BW; ++d) {
        sx += kx[d] * xs[w * RY + r + P][lane + d];
        sy += ky[d] * colv[r + d];
        sz += kz[d] * win[r][d];
      }
      const double v = s * (mJ[r] * mK * sx + mI * mK * sy + mI * mJ[r] * sz);
      y[(int64_t)I + (int64_t)n * Jr[r] + K * n2] = v;
      if constexpr (DOT) dot += win[r][P] * v;
    }
  };
#pragma unroll
  for (int d = 0; d < PD; ++d)
    if (K0 + d < K1) load_plane(K0 + d, treg[d], wnext[d]);
  int K = K0;
  if constexpr (PD == 2) {
    // pairs in the loop (no branch between the halves), an odd last plane after it
    for (; K + 1 < K1; K += 2) {
      plane(K, treg[0], wnext[0]);
      plane(K + 1, treg[1], wnext[1]);
    }
    if (K < K1) plane(K, treg[0], wnext[0]);
  } else {
    for (; K < K1; ++K) plane(K, treg[0], wnext[0]);
  }
  if constexpr (DOT) {
    const double bsum = block_sum(dot, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = bsum;
  }
}

// The two vector passes run by rows of the mesh: wave w of work-group b
// takes the 64 consecutive I of its I-chunk in VR consecutive rows (J, K), so
// the J- and K-dependent factors of diag(A) are wave-uniform and each lane
// keeps its I-dependent ones.  The loads of the partials a pass sums are
// issued first, then all of the rows' loads, so the global sum is formed
// while the rows are in flight.
constexpr int VR = 16;
constexpr int PU = 4;   // partials per thread loaded ahead (the rest, if any, after)
static dim3 vec_grid(int n) {
  const int64_t rows = (int64_t)n * n;
  return dim3((unsigned)(((n + 63) / 64) * ((rows + 4 * VR - 1) / (4 * VR))));
}
struct VecPos {
  int I;           // this lane's node index along x
  int row0;        // first row of the wave's run (row = J + n K < n^2 < 2^31)
  int J0, K0;      // its J and K (wave-uniform)
  bool ilive;
};
__device__ __forceinline__ VecPos vec_pos(int n) {
  const int gx = (n + 63) / 64;
  const int b = (int)blockIdx.x;
  const int bx = b % gx, br = b / gx;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  VecPos v;
  v.I = bx * 64 + ((int)threadIdx.x & 63);
  v.row0 = (br * 4 + w) * VR;
  v.K0 = v.row0 / n;
  v.J0 = v.row0 - v.K0 * n;
  v.ilive = v.I < n;
  return v;
}
// z = r / diag(A) at (I, J, K): the lane's I factors and the row's J, K ones
__device__ __forceinline__ double jacobi_z(double rv, double kdI, double mI, double kdJ, double mJ, double kdK,
                                           double mK, double s) {
  return __dmul_rn(rv, 1.0 / (s * (kdI * mJ * mK + mI * kdJ * mK + mI * mJ * kdK)));
}
// Sum of a[0 .. na) in a fixed order, in two steps: parts_load issues the
// thread's first PU loads, parts_sum adds them, then the rest, then sums over
// the work-group.
__device__ __forceinline__ void parts_load(const double *__restrict__ a, int na, double (&v)[PU]) {
#pragma unroll
  for (int u = 0; u < PU; ++u) {
    const int i = (int)threadIdx.x + u * PB;
    v[u] = i < na ? a[i] : 0.0;
  }
}
__device__ __forceinline__ double parts_sum(const double *__restrict__ a, int na, const double (&v)[PU],
                                            double *sh) {
  double t = 0;
#pragma unroll
  for (int u = 0; u < PU; ++u) t += v[u];
  for (int i = (int)threadIdx.x + PU * PB; i < na; i += PB) t += a[i];
  return block_sum(t, sh);
}

// Iteration it: alpha = r.z / p.q from the product's partials (work-group 0
// keeps it for the direction pass); r -= alpha q; partials of r.z
// (z = r / diag(A)) and r.r.
__global__ __launch_bounds__(PB) void poisson_update_kernel(double *__restrict__ r, const double *__restrict__ q,
                                                            const double *__restrict__ kb,
                                                            const double *__restrict__ m, int n, int p, double s,
                                                            double *__restrict__ scal, int it,
                                                            const double *__restrict__ part_pq, int npq,
                                                            double *__restrict__ part_rz, double *__restrict__ part_rr) {
  __shared__ double sh[PB / 64];
  if (it >= scal[S_STOPAT]) return;
  double pp[PU];
  parts_load(part_pq, npq, pp);
  const int bw = 2 * p + 1;
  const int64_t rows = (int64_t)n * n;
  const VecPos vp = vec_pos(n);
  const double kdI = vp.ilive ? kb[(int64_t)vp.I * bw + p] : 0.0, mI = vp.ilive ? m[vp.I] : 0.0;
  double rv[VR], qv[VR];
#pragma unroll
  for (int u = 0; u < VR; ++u) {
    const int64_t row = vp.row0 + u;
    const bool ok = vp.ilive && row < rows;
    const int64_t idx = vp.I + n * row;
    rv[u] = ok ? r[idx] : 0.0;
    qv[u] = ok ? q[idx] : 0.0;
  }
  const double pq = parts_sum(part_pq, npq, pp, sh);
  const double alpha = pq != 0 ? scal[S_RZ + (it & 1)] / pq : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_ALPHA] = alpha;
  double rz = 0, rr = 0;
  int J = vp.J0, K = vp.K0;
#pragma unroll
  for (int u = 0; u < VR; ++u, ++J) {
    const int64_t row = vp.row0 + u;
    if (row >= rows) break;                         // wave-uniform
    if (J == n) {
      J = 0;
      ++K;
    }
    const double kdJ = kb[(int64_t)J * bw + p], mJ = m[J], kdK = kb[(int64_t)K * bw + p], mK = m[K];
    if (vp.ilive) {
      const int64_t idx = vp.I + n * row;
      const double v = rv[u] - alpha * qv[u];
      r[idx] = v;
      const double zv = jacobi_z(v, kdI, mI, kdJ, mJ, kdK, mK, s);
      rz += v * zv;
      rr += v * v;
    }
  }
  const double a = block_sum(rz, sh);
  const double b = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = a;
    part_rr[blockIdx.x] = b;
  }
}

// Iteration it: r.z' and r.r from the update's partials; x += alpha p (the
// update's alpha); unless r.r meets the tolerance, p = z + beta p with
// z = r / diag(A), beta = r.z' / r.z.  Work-group 0 keeps r.z' (the other
// parity slot), r.r, and the iteration count once the tolerance is met.
__global__ __launch_bounds__(PB) void poisson_dir_kernel(double *__restrict__ x, double *__restrict__ pv,
                                                         const double *__restrict__ r,
                                                         const double *__restrict__ kb,
                                                         const double *__restrict__ m, int n, int p, double s,
                                                         double *__restrict__ scal, int it,
                                                         const double *__restrict__ part_rz,
                                                         const double *__restrict__ part_rr, int nparts) {
  __shared__ double sh[PB / 64];
  if (it >= scal[S_STOPAT]) return;
  double pz[PU], pr[PU];
  parts_load(part_rz, nparts, pz);
  parts_load(part_rr, nparts, pr);
  const double alpha = scal[S_ALPHA], rz_old = scal[S_RZ + (it & 1)], stop = scal[S_STOP];
  const int bw = 2 * p + 1;
  const int64_t rows = (int64_t)n * n;
  const VecPos vp = vec_pos(n);
  const double kdI = vp.ilive ? kb[(int64_t)vp.I * bw + p] : 0.0, mI = vp.ilive ? m[vp.I] : 0.0;
  double pw[VR], rw[VR];
  {
    double xw[VR];
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int64_t row = vp.row0 + u;
      const bool ok = vp.ilive && row < rows;
      const int64_t idx = vp.I + n * row;
      pw[u] = ok ? pv[idx] : 0.0;
      xw[u] = ok ? x[idx] : 0.0;
      rw[u] = ok ? r[idx] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < VR; ++u) {
      const int64_t row = vp.row0 + u;
      if (vp.ilive && row < rows) x[vp.I + n * row] = fma(alpha, pw[u], xw[u]);
    }
  }
  const double rz = parts_sum(part_rz, nparts, pz, sh);
  const double rr = parts_sum(part_rr, nparts, pr, sh);
  const bool last = rr <= stop;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[S_RZ + ((it + 1) & 1)] = rz;
    scal[S_RR] = rr;
    if (last) scal[S_STOPAT] = it + 1;
  }
  if (last) return;
  const double beta = rz_old != 0 ? rz / rz_old : 0.0;
  int J = vp.J0, K = vp.K0;
#pragma unroll
  for (int u = 0; u < VR; ++u, ++J) {
    const int64_t row = vp.row0 + u;
    if (row >= rows) break;                         // wave-uniform
    if (J == n) {
      J = 0;
      ++K;
    }
    if (vp.ilive) {
      const double zv = jacobi_z(rw[u], kdI, mI, kb[(int64_t)J * bw + p], m[J], kb[(int64_t)K * bw + p], m[K], s);
      pv[vp.I + n * row] = fma(beta, pw[u], zv);
    }
  }
}

// Setup: r = f - A x (q = A x given), p = z = r / diag(A); partials of r.z,
// r.r and f.f.
__global__ __launch_bounds__(PB) void poisson_init_kernel(const double *__restrict__ f, const double *__restrict__ q,
                                                          double *__restrict__ r, double *__restrict__ pv,
                                                          const double *__restrict__ kb,
                                                          const double *__restrict__ m, int n, int p, double s,
                                                          double *__restrict__ part_rz, double *__restrict__ part_rr,
                                                          double *__restrict__ part_ff) {
  __shared__ double sh[PB];
  const int64_t nd = (int64_t)n * n * n;
  const int bw = 2 * p + 1;
  double rz = 0, rr = 0, ff = 0;
  for (int64_t idx = (int64_t)blockIdx.x * PB + threadIdx.x; idx < nd; idx += (int64_t)gridDim.x * PB) {
    const double fv = f[idx];
    const double rv = fv - q[idx];
    const int I = (int)(idx % n), J = (int)((idx / n) % n), K = (int)(idx / ((int64_t)n * n));
    const double zv = jacobi_z(rv, kb[(int64_t)I * bw + p], m[I], kb[(int64_t)J * bw + p], m[J],
                               kb[(int64_t)K * bw + p], m[K], s);
    r[idx] = rv;
    pv[idx] = zv;
    rz += rv * zv;
    rr += rv * rv;
    ff += fv * fv;
  }
  const double a = block_sum(rz, sh);
  const double b = block_sum(rr, sh);
  const double c = block_sum(ff, sh);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = a;
    part_rr[blockIdx.x] = b;
    part_ff[blockIdx.x] = c;
  }
}

// f = M rho, M = 1 / minv^2
__global__ __launch_bounds__(PB) void poisson_rhs_kernel(const double *__restrict__ rho,
                                                         const double *__restrict__ minv, double *__restrict__ f,
                                                         int64_t nd) {
  for (int64_t idx = (int64_t)blockIdx.x * PB + threadIdx.x; idx < nd; idx += (int64_t)gridDim.x * PB)
    f[idx] = rho[idx] / (minv[idx] * minv[idx]);
}

// point charges on their nodes (distinct dofs)
__global__ __launch_bounds__(PB) void poisson_charges_kernel(double *__restrict__ f, const int64_t *__restrict__ dofs,
                                                             const double *__restrict__ q, int nq) {
  const int i = blockIdx.x * PB + threadIdx.x;
  if (i < nq) f[dofs[i]] += q[i];
}

// Setup sums in a fixed order: r.z (the slot of iteration 0), r.r, f.f; the
// stop threshold tol^2 f.f and the stop count (0 when the initial guess
// already meets the tolerance).
__global__ __launch_bounds__(PR) void poisson_setup_reduce_kernel(const double *__restrict__ a,
                                                                  const double *__restrict__ b,
                                                                  const double *__restrict__ c, int nparts,
                                                                  double tol2, double *__restrict__ scal) {
  __shared__ double sh[PR];
  double sa = 0, sb = 0, sc = 0;
  for (int i = threadIdx.x; i < nparts; i += PR) {
    sa += a[i];
    sb += b[i];
    sc += c[i];
  }
  sa = block_sum<PR>(sa, sh);
  sb = block_sum<PR>(sb, sh);
  sc = block_sum<PR>(sc, sh);
  if (threadIdx.x == 0) {
    scal[S_RZ] = sa;
    scal[S_RZ + 1] = 0.0;
    scal[S_RR] = sb;
    scal[S_FF] = sc;
    scal[S_STOP] = tol2 * sc;
    scal[S_ALPHA] = 0.0;
    scal[S_STOPAT] = sb <= tol2 * sc ? 0.0 : kNever;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// 1D Laplacian stiffness (band, half-width p) and GLL mass on the interior
// nodes, assembled from the reference matrices.
static void poisson_tables(const MeshTables &M, std::vector<double> &kb, std::vector<double> &m1) {
  const int p = M.p, q = M.q, n = M.n, n1 = M.n_el * p + 1, bw = 2 * p + 1;
  std::vector<double> K((size_t)n1 * n1, 0.0), mm(n1, 0.0);
  for (int e = 0; e < M.n_el; ++e)
    for (int a = 0; a < q; ++a) {
      mm[e * p + a] += (M.h / 2.0) * M.w[a];
      for (int b = 0; b < q; ++b) K[(size_t)(e * p + a) * n1 + (e * p + b)] += (2.0 / M.h) * M.K1[(size_t)a * q + b];
    }
  kb.assign((size_t)n * bw, 0.0);
  m1.resize(n);
  for (int i = 0; i < n; ++i) {
    m1[i] = mm[i + 1];
    for (int d = -p; d <= p; ++d) {
      const int j = i + d;
      if (j >= 0 && j < n) kb[(size_t)i * bw + d + p] = K[(size_t)(i + 1) * n1 + (j + 1)];
    }
  }
}

static int poisson_ready(chfsi_ctx *c) {
  if (!c) return CHFSI_ERR_ARG;
  if (c->device < 0) return fail(c, CHFSI_ERR_STATE, "host-only context: no device work");
  if (!c->has_mesh) return fail(c, CHFSI_ERR_STATE, "poisson: set_mesh first");
  if (c->mesh.periodic)
    return fail(c, CHFSI_ERR_STATE, "poisson: the periodic cell needs a neutral charge (not supported)");
  if (int r = set_dev(c)) return r;
  const MeshTables &M = c->mesh;
  const size_t bw = 2 * M.p + 1;
  if (c->pois_n != M.n || c->pois_p != M.p || c->pois_h != M.h) {
    std::vector<double> kb, m1;
    poisson_tables(M, kb, m1);
    HIPCHK(c, c->pois_kb.ensure(kb.size() * sizeof(double)));
    HIPCHK(c, c->pois_m.ensure(m1.size() * sizeof(double)));
    HIPCHK(c, hipMemcpyAsync(c->pois_kb.p, kb.data(), (size_t)M.n * bw * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->pois_m.p, m1.data(), m1.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->pois_n = M.n;
    c->pois_p = M.p;
    c->pois_h = M.h;
  }
  return 0;
}

static const double kInv4Pi = 0.25 / 3.14159265358979323846;

// stencil tile: rows per wave, planes per work-group, planes loaded ahead
// (measured at the 143^3 and 159^3 interior meshes)
constexpr int POIS_RY = 2, POIS_KB = 8, POIS_PD = 1;

static dim3 apply_grid(int n) {
  constexpr int TY = 4 * POIS_RY;
  return dim3((unsigned)((n + TX - 1) / TX) * ((n + TY - 1) / TY) * ((n + POIS_KB - 1) / POIS_KB));
}

// y = A x; with part (and scal, it): the partials of x . y for iteration it
// (skipped once the solve has stopped).  -1 for an unsupported degree.
static int poisson_stencil_launch(const MeshTables &M, const double *x, double *y, const double *kb, const double *m,
                                  const double *scal, int it, double *part, hipStream_t s) {
  const dim3 g = apply_grid(M.n), b(PB);
  switch (M.p) {
#define CHFSI_POIS_P(P)                                                                                        \
  case P:                                                                                                      \
    if (part)                                                                                                  \
      hipLaunchKernelGGL((poisson_stencil_kernel<P, POIS_RY, POIS_KB, POIS_PD, true>), g, b, 0, s, x, y, kb, m, M.n,       \
                         kInv4Pi, scal, it, part);                                                                 \
    else                                                                                                       \
      hipLaunchKernelGGL((poisson_stencil_kernel<P, POIS_RY, POIS_KB, POIS_PD, false>), g, b, 0, s, x, y, kb, m, M.n,      \
                         kInv4Pi, nullptr, 0, nullptr);                                                           \
    return 0;
    CHFSI_POIS_P(1) CHFSI_POIS_P(2) CHFSI_POIS_P(3) CHFSI_POIS_P(4) CHFSI_POIS_P(5) CHFSI_POIS_P(6)
    CHFSI_POIS_P(7)
#undef CHFSI_POIS_P
    default: return -1;
  }
}

}  // namespace chfsi

using namespace chfsi;

extern "C" int chfsi_poisson_apply(chfsi_ctx *c, const double *x, double *y) {
  if (int r = poisson_ready(c)) return r;
  if (!x || !y || x == y) return fail(c, CHFSI_ERR_ARG, "poisson_apply: x and y must be separate device arrays");
  if (poisson_stencil_launch(c->mesh, x, y, c->pois_kb.as<double>(), c->pois_m.as<double>(), nullptr, 0, nullptr,
                             c->stream))
    return fail(c, CHFSI_ERR_ARG, "poisson_apply: degree p must be in 1..7");
  HIPCHK(c, hipGetLastError());
  return 0;
}

extern "C" int chfsi_poisson_solve(chfsi_ctx *c, const double *rho, int ncharges, const int64_t *charge_dofs,
                                   const double *charges, double *phi, double tol, int max_iter, int *iters,
                                   double *rel_resid) {
  if (int r = poisson_ready(c)) return r;
  const MeshTables &M = c->mesh;
  const int64_t nd = M.n_dof;
  if (!rho || !phi || !(tol > 0) || max_iter < 0 || ncharges < 0 || (ncharges > 0 && (!charge_dofs || !charges)))
    return fail(c, CHFSI_ERR_ARG, "poisson_solve: bad arguments");
  if (M.p < 1 || M.p > 7) return fail(c, CHFSI_ERR_ARG, "poisson_solve: degree p must be in 1..7");
  // point charges: combined per node on the host, so the device adds each once
  std::map<int64_t, double> qmap;
  for (int i = 0; i < ncharges; ++i) {
    if (charge_dofs[i] < 0 || charge_dofs[i] >= nd || !std::isfinite(charges[i]))
      return fail(c, CHFSI_ERR_ARG, "poisson_solve: charge dof out of range or non-finite charge");
    qmap[charge_dofs[i]] += charges[i];
  }
  const int64_t nb = std::min<int64_t>((nd + PB - 1) / PB, MAXG);   // element-wise grids (grid-stride)
  const int64_t nv = vec_grid(M.n).x;                // the two vector passes
  const dim3 ga = apply_grid(M.n);
  const int64_t na = (int64_t)ga.x * ga.y * ga.z;  // product grid
  const int64_t npart = std::max(std::max(nb, na), nv);
  // workspace: f, r, p, q (nd each), partials (3 npart), scalars
  HIPCHK(c, c->pois_work.ensure((size_t)(4 * nd + 3 * npart + S_NSCAL) * sizeof(double)));
  double *f = c->pois_work.as<double>(), *r = f + nd, *pv = r + nd, *q = pv + nd;
  double *pa = q + nd, *pb = pa + npart, *pc = pb + npart, *scal = pc + npart;
  const double *kb = c->pois_kb.as<double>(), *m = c->pois_m.as<double>();
  const dim3 grid((unsigned)nb), block(PB);
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(poisson_rhs_kernel, grid, block, 0, s, rho, c->minv64.as<double>(), f, nd);
  if (!qmap.empty()) {
    std::vector<int64_t> qd;
    std::vector<double> qv;
    for (auto &e : qmap) {
      qd.push_back(e.first);
      qv.push_back(e.second);
    }
    HIPCHK(c, c->pois_q.ensure(qd.size() * (sizeof(int64_t) + sizeof(double))));
    int64_t *dq = c->pois_q.as<int64_t>();
    double *vq = reinterpret_cast<double *>(dq + qd.size());
    HIPCHK(c, hipMemcpyAsync(dq, qd.data(), qd.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(vq, qv.data(), qv.size() * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(poisson_charges_kernel, dim3((unsigned)((qd.size() + PB - 1) / PB)), block, 0, s, f, dq, vq,
                       (int)qd.size());
    HIPCHK(c, hipStreamSynchronize(s));            // the host staging vectors go out of scope
  }
  poisson_stencil_launch(M, phi, q, kb, m, nullptr, 0, nullptr, s);
  hipLaunchKernelGGL(poisson_init_kernel, grid, block, 0, s, f, q, r, pv, kb, m, M.n, M.p, kInv4Pi, pa, pb, pc);
  hipLaunchKernelGGL(poisson_setup_reduce_kernel, dim3(1), dim3(PR), 0, s, pa, pb, pc, (int)nb, tol * tol, scal);
  // iterations in groups; the device records the iteration that met the
  // tolerance, the host reads it between groups (a group started after the
  // stop costs only its empty launches)
  constexpr int GROUP = 8;
  double hs[S_NSCAL];
  int launched = 0;
  while (launched < max_iter) {
    const int k = std::min(GROUP, max_iter - launched);
    for (int i = 0; i < k; ++i, ++launched) {
      poisson_stencil_launch(M, pv, q, kb, m, scal, launched, pc, s);
      hipLaunchKernelGGL(poisson_update_kernel, dim3((unsigned)nv), block, 0, s, r, q, kb, m, M.n, M.p, kInv4Pi, scal,
                         launched, pc, (int)na, pa, pb);
      hipLaunchKernelGGL(poisson_dir_kernel, dim3((unsigned)nv), block, 0, s, phi, pv, r, kb, m, M.n, M.p, kInv4Pi,
                         scal, launched, pa, pb, (int)nv);
    }
    HIPCHK(c, hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (hs[S_STOPAT] <= launched) break;
  }
  HIPCHK(c, hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const int it = hs[S_STOPAT] < launched ? (int)hs[S_STOPAT] : launched;
  // the true residual of the returned phi
  poisson_stencil_launch(M, phi, q, kb, m, nullptr, 0, nullptr, s);
  hipLaunchKernelGGL(poisson_init_kernel, grid, block, 0, s, f, q, r, pv, kb, m, M.n, M.p, kInv4Pi, pa, pb, pc);
  hipLaunchKernelGGL(poisson_setup_reduce_kernel, dim3(1), dim3(PR), 0, s, pa, pb, pc, (int)nb, tol * tol, scal);
  HIPCHK(c, hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  HIPCHK(c, hipGetLastError());
  if (iters) *iters = it;
  const double ff = hs[S_FF];
  const double res = ff > 0 ? std::sqrt(hs[S_RR] / ff) : 0.0;
  if (rel_resid) *rel_resid = res;
  return res <= tol ? 0 : CHFSI_WARN_NOT_CONVERGED;
}
