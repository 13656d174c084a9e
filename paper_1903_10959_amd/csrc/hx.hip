// Chebyshev-step kernels: Y = s1 (Htilde - shift) X + s2 Xprev with
// Htilde X = M^-1/2 (sum_e P_e^T K_e P_e) M^-1/2 X + V .* X.
//
// Paper, Sec. 3.3 (practical implementation of Chebyshev filtering): store the
// cell Hamiltonian, extract the cell wavefunction matrices from the DoF-major
// global block, multiply, assemble.  On a uniform mesh every cell carries the
// same stiffness K_ref, so the cell products form one dense contraction
// K_ref [n_loc x n_loc] x X_e [n_loc x ncols] per cell, done here on MFMA.
// Under GLL quadrature the potential part is diagonal.
//
// Assembly is atomic-free: cells are launched colour by colour (8 colours,
// (ex&1)+2(ey&1)+4(ez&1)); cells of one colour share no DoF, so each output
// row is touched by exactly one work-group per launch.  The element-wise part
// s1 (V - shift) X + s2 Xprev is fused into the first touch: colours run in
// increasing order, and the first colour containing a node is the one whose
// parity bit is 0 in every direction where the node lies on a cell face; the
// single cell of that colour containing the node writes Y (element-wise part
// plus its product), every later cell adds to Y.
#include "common.hpp"
#include "kernels.hpp"

namespace chfsi {

// ---------------------------------------------------------------------------
// Cell products of one colour.  Work-group = one cell x 64 columns; wave w owns
// columns [n0, n0+16) with n0 = 64*tile + 16*w.  The cell's dof indices and
// M^-1/2 values are staged in LDS, so the B operand (gathered, M^-1/2-scaled
// X rows, 16 contiguous values per row) costs one LDS read and one global load
// with no data-dependent branch.  A operand: K_ref (symmetric, zero padded to
// NP) read row-wise, A[i][k] = K[k][i] contiguous in i.  Output row blocks are
// processed RBP at a time so the accumulators stay in registers.
// Epilogue: Y[dof, col] += s1 * minv[dof] * acc.
// ---------------------------------------------------------------------------
template <typename T, int NP>
struct CellTile {
  static constexpr int RB = NP / 16;
  // FP64 accumulators are 8 registers per 16x16 block: at most 11 blocks live
  static constexpr int RBP = sizeof(T) == 8 ? (RB % 11 == 0 ? 11 : (RB % 8 == 0 ? 8 : (RB % 7 == 0 ? 7 : RB)))
                                            : RB;
  static_assert(RB % RBP == 0, "row-block pass must divide the row blocks");
};

// 1 when this cell is the first (in colour order) to touch local node r
__device__ __forceinline__ int first_touch(int r, int q, int e, int n_el) {
  const int a = r % q, b = (r / q) % q, c = r / (q * q);
  const int ex = e % n_el, ey = (e / n_el) % n_el, ez = e / (n_el * n_el);
  const bool fx = (a > 0 && a < q - 1) || !(ex & 1);
  const bool fy = (b > 0 && b < q - 1) || !(ey & 1);
  const bool fz = (c > 0 && c < q - 1) || !(ez & 1);
  return (fx && fy && fz) ? 1 : 0;
}

// The product of one cell and one 64-column tile (called by the single-problem
// and the batched kernels).
template <typename T, int NP>
__device__ __forceinline__ void cell_tile(const T *__restrict__ X, int64_t ldx, const T *__restrict__ Xp,
                                          int64_t ldp, T *__restrict__ Y, int64_t ldy, const T *__restrict__ K,
                                          const int32_t *__restrict__ cmap, int n_loc, int q, int n_el, int e,
                                          int tile, const T *__restrict__ minv, const T *__restrict__ V, int ncols,
                                          T s1, T s2, T shift) {
  typedef typename acc4<T>::type acc_t;
  constexpr int RB = CellTile<T, NP>::RB;
  constexpr int RBP = CellTile<T, NP>::RBP;
  __shared__ int32_t dof_s[NP];
  __shared__ T mi_s[NP];
  __shared__ T vd_s[NP];     // s1 (V - shift) on first-touch rows
  __shared__ int8_t ft_s[NP];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int r = threadIdx.x; r < NP; r += blockDim.x) {
    int d = r < n_loc ? cmap[(int64_t)e * n_loc + r] : -1;
    dof_s[r] = d < 0 ? 0 : d;              // clamped: row 0 is always readable
    mi_s[r] = d < 0 ? T(0) : minv[d];      // zero weight removes Dirichlet / padding rows
    const int ft = d < 0 ? 0 : first_touch(r, q, e, n_el);
    ft_s[r] = (int8_t)ft;
    vd_s[r] = ft ? s1 * (V[d] - shift) : T(0);
  }
  __syncthreads();
  const int j = lane & 15, kq = lane >> 4;
  const int col = tile * 64 + wave * 16 + j;
  const bool col_ok = col < ncols;
  const int colc = col_ok ? col : ncols - 1;   // clamped column, in bounds
  const T cscale = col_ok ? T(1) : T(0);

#pragma unroll 1
  for (int rb0 = 0; rb0 < RB; rb0 += RBP) {
    acc_t acc[RBP];
#pragma unroll
    for (int r = 0; r < RBP; ++r) acc[r] = acc_t{0, 0, 0, 0};
    const T *__restrict__ Kp = K + kq * NP + rb0 * 16 + j;

    // two operand sets in ping-pong: the loads of step k+1 are in flight while
    // the MFMAs of step k issue (NP/4 is even for every NP used)
    auto load_b = [&](int k) -> T {
      const int row = 4 * k + kq;
      return X[(int64_t)dof_s[row] * ldx + colc] * (mi_s[row] * cscale);
    };
    T b0 = load_b(0), b1;
    T a0[RBP], a1[RBP];
#pragma unroll
    for (int r = 0; r < RBP; ++r) a0[r] = Kp[r * 16];

#pragma unroll 1
    for (int k = 0; k < NP / 4; k += 2) {
      b1 = load_b(k + 1);
#pragma unroll
      for (int r = 0; r < RBP; ++r) a1[r] = Kp[(int64_t)(4 * (k + 1)) * NP + r * 16];
#pragma unroll
      for (int r = 0; r < RBP; ++r) acc[r] = mfma16x4(a0[r], b0, acc[r]);
      const int k2 = (k + 2 < NP / 4) ? k + 2 : k;   // last pair re-reads step k (in bounds, unused)
      b0 = load_b(k2);
#pragma unroll
      for (int r = 0; r < RBP; ++r) a0[r] = Kp[(int64_t)(4 * k2) * NP + r * 16];
#pragma unroll
      for (int r = 0; r < RBP; ++r) acc[r] = mfma16x4(a1[r], b1, acc[r]);
    }

    if (col_ok) {
      if (sizeof(T) == 4) {
        // FP32: epilogue in chunks of 4 row blocks, every load of a chunk issued
        // before its stores (16 rows per lane in flight; measured faster)
#pragma unroll
        for (int r0 = 0; r0 < RBP; r0 += 4) {
          T old[4][4];
#pragma unroll
          for (int r = r0; r < r0 + 4 && r < RBP; ++r)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
              const int row = (rb0 + r) * 16 + acc_row<T>(kq, qq);
              T v = T(0);
              if (row < n_loc && mi_s[row] != T(0)) {
                const int64_t d = dof_s[row];
                if (ft_s[row]) {
                  v = vd_s[row] * X[d * ldx + col];
                  if (Xp) v += s2 * Xp[d * ldp + col];
                } else {
                  v = Y[d * ldy + col];
                }
              }
              old[r - r0][qq] = v;
            }
#pragma unroll
          for (int r = r0; r < r0 + 4 && r < RBP; ++r)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
              const int row = (rb0 + r) * 16 + acc_row<T>(kq, qq);
              if (row < n_loc) {
                const T w = mi_s[row];
                if (w != T(0)) Y[(int64_t)dof_s[row] * ldy + col] = old[r - r0][qq] + s1 * w * acc[r][qq];
              }
            }
        }
      } else {
        // FP64 (compute-bound): row by row; other work-groups on the CU hide the latency
#pragma unroll
        for (int r = 0; r < RBP; ++r)
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int row = (rb0 + r) * 16 + acc_row<T>(kq, qq);
            if (row < n_loc) {
              const T w = mi_s[row];
              if (w != T(0)) {
                const int64_t d = dof_s[row];
                T *yp = Y + d * ldy + col;
                const T prod = s1 * w * acc[r][qq];
                if (ft_s[row]) {
                  T y = vd_s[row] * X[d * ldx + col] + prod;
                  if (Xp) y += s2 * Xp[d * ldp + col];
                  *yp = y;
                } else {
                  *yp += prod;
                }
              }
            }
          }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 cell products (FP32 state, FP32 accumulation): v_mfma_f32_16x16x32_bf16.
// The cell's gathered, M^-1/2-scaled X rows (64 columns) are converted to BF16
// (round to nearest even) and staged in LDS transposed, [column][local node],
// so a B fragment (8 consecutive local nodes of one column) is one 16-byte LDS
// read.  SPLIT: X = hi + lo and K = hi + lo in BF16, three products
// hi*hi + hi*lo + lo*hi accumulated in FP32.  NPB: n_loc rounded up to 32.
// ---------------------------------------------------------------------------
template <int NPB, bool SPLIT>
__global__ __launch_bounds__(256) void hx_cells_bf16_kernel(const float *__restrict__ X, int64_t ldx,
                                                            const float *__restrict__ Xp, int64_t ldp,
                                                            float *__restrict__ Y, int64_t ldy,
                                                            const __bf16 *__restrict__ Kh,
                                                            const __bf16 *__restrict__ Kl,
                                                            const int32_t *__restrict__ cmap, int n_loc, int q,
                                                            int n_el, const int32_t *__restrict__ cells,
                                                            const float *__restrict__ minv,
                                                            const float *__restrict__ V, int ncols, int ntiles,
                                                            float s1, float s2, float shift) {
  constexpr int RB = NPB / 16;
  constexpr int LDX = NPB + 8;            // row of the transposed tile, 16-byte aligned
  constexpr int NPART = SPLIT ? 2 : 1;
  __shared__ int32_t dof_s[NPB];
  __shared__ float mi_s[NPB];
  __shared__ float vd_s[NPB];
  __shared__ int8_t ft_s[NPB];
  __shared__ __attribute__((aligned(16))) __bf16 xs[NPART][64 * LDX];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cell_slot = blockIdx.x / ntiles;
  const int tile = blockIdx.x - cell_slot * ntiles;
  const int e = cells[cell_slot];
  const int col0 = tile * 64;
  for (int r = threadIdx.x; r < NPB; r += blockDim.x) {
    int d = r < n_loc ? cmap[(int64_t)e * n_loc + r] : -1;
    dof_s[r] = d < 0 ? 0 : d;
    mi_s[r] = d < 0 ? 0.f : minv[d];
    const int ft = d < 0 ? 0 : first_touch(r, q, e, n_el);
    ft_s[r] = (int8_t)ft;
    vd_s[r] = ft ? s1 * (V[d] - shift) : 0.f;
  }
  __syncthreads();
  // stage: 4 consecutive columns per thread per row (16-byte global loads when
  // aligned), SU rows per thread per round with every load issued first
  const bool vec_ok = ((ldx & 3) == 0) && ((col0 & 3) == 0) && ((((uintptr_t)X) & 15) == 0);
  constexpr int SU = 8;
  for (int base = threadIdx.x; base < NPB * 16; base += SU * 256) {
    float v[SU][4];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int idx = base + u * 256;
      v[u][0] = v[u][1] = v[u][2] = v[u][3] = 0.f;
      if (idx < NPB * 16) {
        const int r = idx >> 4, c4 = (idx & 15) * 4;
        const float *src = X + (int64_t)dof_s[r] * ldx + col0 + c4;
        if (vec_ok && col0 + c4 + 3 < ncols) {
          const float4 t = *reinterpret_cast<const float4 *>(src);
          v[u][0] = t.x; v[u][1] = t.y; v[u][2] = t.z; v[u][3] = t.w;
        } else {
#pragma unroll
          for (int w = 0; w < 4; ++w) v[u][w] = (col0 + c4 + w < ncols) ? src[w] : 0.f;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int idx = base + u * 256;
      if (idx < NPB * 16) {
        const int r = idx >> 4, c4 = (idx & 15) * 4;
        const float w = mi_s[r];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float x = v[u][t] * w;
          const __bf16 h = (__bf16)x;
          xs[0][(c4 + t) * LDX + r] = h;
          if (SPLIT) xs[NPART - 1][(c4 + t) * LDX + r] = (__bf16)(x - (float)h);
        }
      }
    }
  }
  __syncthreads();
  const int j = lane & 15, kq = lane >> 4;
  const int lcol = wave * 16 + j;               // column within the tile
  const int col = col0 + lcol;
  v4f acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = v4f{0, 0, 0, 0};
  typedef __attribute__((ext_vector_type(4))) int v4i;
  for (int k = 0; k < NPB; k += 32) {
    const int kk = k + 8 * kq;
    v8bf bh, bl;
    {
      v4i t = *reinterpret_cast<const v4i *>(&xs[0][lcol * LDX + kk]);
      bh = __builtin_bit_cast(v8bf, t);
      if (SPLIT) {
        v4i t2 = *reinterpret_cast<const v4i *>(&xs[NPART - 1][lcol * LDX + kk]);
        bl = __builtin_bit_cast(v8bf, t2);
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      // A[i][k..k+7] = K[i][k..k+7] (row i = 16 r + j): one 16-byte load
      const v4i ta = *reinterpret_cast<const v4i *>(Kh + (int64_t)(r * 16 + j) * NPB + kk);
      const v8bf ah = __builtin_bit_cast(v8bf, ta);
      acc[r] = mfma16x32bf(ah, bh, acc[r]);
      if (SPLIT) {
        const v4i tl = *reinterpret_cast<const v4i *>(Kl + (int64_t)(r * 16 + j) * NPB + kk);
        const v8bf al = __builtin_bit_cast(v8bf, tl);
        acc[r] = mfma16x32bf(ah, bl, acc[r]);
        acc[r] = mfma16x32bf(al, bh, acc[r]);
      }
    }
  }
  if (col >= ncols) return;
#pragma unroll
  for (int r0 = 0; r0 < RB; r0 += 4) {
    float old[4][4];
#pragma unroll
    for (int r = r0; r < r0 + 4 && r < RB; ++r)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int row = r * 16 + acc_row<float>(kq, qq);
        float v = 0.f;
        if (row < n_loc && mi_s[row] != 0.f) {
          const int64_t d = dof_s[row];
          if (ft_s[row]) {
            v = vd_s[row] * X[d * ldx + col];
            if (Xp) v += s2 * Xp[d * ldp + col];
          } else {
            v = Y[d * ldy + col];
          }
        }
        old[r - r0][qq] = v;
      }
#pragma unroll
    for (int r = r0; r < r0 + 4 && r < RB; ++r)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int row = r * 16 + acc_row<float>(kq, qq);
        if (row < n_loc) {
          const float w = mi_s[row];
          if (w != 0.f) Y[(int64_t)dof_s[row] * ldy + col] = old[r - r0][qq] + s1 * w * acc[r][qq];
        }
      }
  }
}

template <int NPB, bool SPLIT>
static void launch_bf16(const HxBf16Args &a, int color_begin, int color_end, hipStream_t s) {
  int ntiles = (a.ncols + 63) / 64;
  int ncell = color_end - color_begin;
  if (ncell <= 0 || ntiles <= 0) return;
  hipLaunchKernelGGL((hx_cells_bf16_kernel<NPB, SPLIT>), dim3((unsigned)(ncell * ntiles)), dim3(256), 0, s, a.X,
                     a.ldx, a.Xp, a.ldp, a.Y, a.ldy, a.Kh, a.Kl, a.cmap, a.n_loc, a.q, a.n_el,
                     a.cells + color_begin, a.minv, a.V, a.ncols, ntiles, a.s1, a.s2, a.shift);
}

template <bool SPLIT>
static int dispatch_bf16(const HxBf16Args &a, int cb, int ce, hipStream_t s) {
  switch (a.npb) {
    case 32: launch_bf16<32, SPLIT>(a, cb, ce, s); break;
    case 64: launch_bf16<64, SPLIT>(a, cb, ce, s); break;
    case 128: launch_bf16<128, SPLIT>(a, cb, ce, s); break;
    case 224: launch_bf16<224, SPLIT>(a, cb, ce, s); break;
    case 352: launch_bf16<352, SPLIT>(a, cb, ce, s); break;
    case 512: launch_bf16<512, SPLIT>(a, cb, ce, s); break;
    default: return -1;
  }
  return 0;
}

int hx_cells_bf16_launch(const HxBf16Args &a, int color_begin, int color_end, hipStream_t s) {
  return a.split ? dispatch_bf16<true>(a, color_begin, color_end, s) : dispatch_bf16<false>(a, color_begin, color_end, s);
}

template <typename T, int NP>
__global__ __launch_bounds__(256) void hx_cells_kernel(const T *__restrict__ X, int64_t ldx,
                                                       const T *__restrict__ Xp, int64_t ldp,
                                                       T *__restrict__ Y, int64_t ldy,
                                                       const T *__restrict__ K,
                                                       const int32_t *__restrict__ cmap, int n_loc,
                                                       int q, int n_el,
                                                       const int32_t *__restrict__ cells,
                                                       const T *__restrict__ minv, const T *__restrict__ V,
                                                       int ncols, int ntiles, T s1, T s2, T shift) {
  const int cell_slot = blockIdx.x / ntiles;
  const int tile = blockIdx.x - cell_slot * ntiles;
  cell_tile<T, NP>(X, ldx, Xp, ldp, Y, ldy, K, cmap, n_loc, q, n_el, cells[cell_slot], tile, minv, V, ncols, s1, s2,
                   shift);
}

// Batched: work item = (problem, cell, column tile); the step's buffer roles
// (input, previous, output) are the same for every problem, its coefficients
// come from the problem's table (s1, s2, shift per step).
template <typename T, int NP>
__global__ __launch_bounds__(256) void hx_cells_batch_kernel(const BatchProblem<T> *__restrict__ probs,
                                                             const int4 *__restrict__ work, int step, int cur,
                                                             int prev, int out) {
  const int4 w = work[blockIdx.x];
  const BatchProblem<T> &P = probs[w.x];
  const T *coef = P.coef + 3 * step;
  cell_tile<T, NP>(P.buf[cur], P.ld[cur], prev >= 0 ? P.buf[prev] : nullptr, prev >= 0 ? P.ld[prev] : 0,
                   P.buf[out], P.ld[out], P.K, P.cmap, P.n_loc, P.q, P.n_el, w.y, w.z, P.minv, P.V, P.ncols,
                   coef[0], coef[1], coef[2]);
}

template <typename T, int NP>
static void launch_batch(const BatchProblem<T> *probs, const int4 *work, int nwork, int step, int cur, int prev,
                         int out, hipStream_t s) {
  if (nwork <= 0) return;
  hipLaunchKernelGGL((hx_cells_batch_kernel<T, NP>), dim3((unsigned)nwork), dim3(256), 0, s, probs, work, step, cur,
                     prev, out);
}

template <typename T>
int hx_cells_batch_launch(int np, const BatchProblem<T> *probs, const int4 *work, int nwork, int step, int cur,
                          int prev, int out, hipStream_t s) {
  switch (np) {
    case 16: launch_batch<T, 16>(probs, work, nwork, step, cur, prev, out, s); break;
    case 32: launch_batch<T, 32>(probs, work, nwork, step, cur, prev, out, s); break;
    case 64: launch_batch<T, 64>(probs, work, nwork, step, cur, prev, out, s); break;
    case 128: launch_batch<T, 128>(probs, work, nwork, step, cur, prev, out, s); break;
    case 224: launch_batch<T, 224>(probs, work, nwork, step, cur, prev, out, s); break;
    case 352: launch_batch<T, 352>(probs, work, nwork, step, cur, prev, out, s); break;
    case 512: launch_batch<T, 512>(probs, work, nwork, step, cur, prev, out, s); break;
    default: return -1;
  }
  return 0;
}
template int hx_cells_batch_launch<double>(int, const BatchProblem<double> *, const int4 *, int, int, int, int, int,
                                           hipStream_t);
template int hx_cells_batch_launch<float>(int, const BatchProblem<float> *, const int4 *, int, int, int, int, int,
                                          hipStream_t);

template <typename T, int NP>
static void launch_cells(const HxArgs<T> &a, int color_begin, int color_end, hipStream_t s) {
  int ntiles = (a.ncols + 63) / 64;
  int ncell = color_end - color_begin;
  if (ncell <= 0 || ntiles <= 0) return;
  dim3 grid((unsigned)(ncell * ntiles)), block(256);
  hipLaunchKernelGGL((hx_cells_kernel<T, NP>), grid, block, 0, s, a.X, a.ldx, a.Xp, a.ldp, a.Y, a.ldy, a.K,
                     a.cmap, a.n_loc, a.q, a.n_el, a.cells + color_begin, a.minv, a.V, a.ncols, ntiles, a.s1, a.s2,
                     a.shift);
}

template <typename T>
int hx_cells_launch(const HxArgs<T> &a, int color_begin, int color_end, hipStream_t s) {
  switch (a.np) {
    case 16: launch_cells<T, 16>(a, color_begin, color_end, s); break;    // p = 1
    case 32: launch_cells<T, 32>(a, color_begin, color_end, s); break;    // p = 2
    case 64: launch_cells<T, 64>(a, color_begin, color_end, s); break;    // p = 3
    case 128: launch_cells<T, 128>(a, color_begin, color_end, s); break;  // p = 4
    case 224: launch_cells<T, 224>(a, color_begin, color_end, s); break;  // p = 5
    case 352: launch_cells<T, 352>(a, color_begin, color_end, s); break;  // p = 6
    case 512: launch_cells<T, 512>(a, color_begin, color_end, s); break;  // p = 7
    default: return -1;
  }
  return 0;
}

template int hx_cells_launch<double>(const HxArgs<double> &, int, int, hipStream_t);
template int hx_cells_launch<float>(const HxArgs<float> &, int, int, hipStream_t);
// ---------------------------------------------------------------------------
// Precision conversion and column-block copies (strided, DoF-major)
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void copy_cols_kernel(const Tin *__restrict__ in, int64_t ldi,
                                                        Tout *__restrict__ out, int64_t ldo, int64_t nrows,
                                                        int ncols) {
  const int64_t total = nrows * (int64_t)ncols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / ncols;
    int j = (int)(t - i * ncols);
    out[i * ldo + j] = (Tout)in[i * ldi + j];
  }
}

template <typename Tin, typename Tout>
void copy_cols_launch(const Tin *in, int64_t ldi, Tout *out, int64_t ldo, int64_t nrows, int ncols,
                      hipStream_t s) {
  int64_t total = nrows * ncols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return;
  hipLaunchKernelGGL((copy_cols_kernel<Tin, Tout>), dim3((unsigned)blocks), dim3(256), 0, s, in, ldi, out, ldo,
                     nrows, ncols);
}
template void copy_cols_launch<double, double>(const double *, int64_t, double *, int64_t, int64_t, int,
                                               hipStream_t);
template void copy_cols_launch<double, float>(const double *, int64_t, float *, int64_t, int64_t, int,
                                              hipStream_t);
template void copy_cols_launch<float, double>(const float *, int64_t, double *, int64_t, int64_t, int,
                                              hipStream_t);
template void copy_cols_launch<float, float>(const float *, int64_t, float *, int64_t, int64_t, int, hipStream_t);

// Sets *flag = 1 if any of the nrows x ncols values is NaN or Inf.
template <typename T>
__global__ __launch_bounds__(256) void nonfinite_kernel(const T *__restrict__ X, int64_t ld, int64_t nrows,
                                                        int ncols, int *flag) {
  const int64_t total = nrows * (int64_t)ncols;
  bool bad = false;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / ncols;
    int j = (int)(t - i * ncols);
    T v = X[i * ld + j];
    if (!(v - v == T(0))) bad = true;
  }
  if (bad) *flag = 1;
}

template <typename T>
void nonfinite_launch(const T *X, int64_t ld, int64_t nrows, int ncols, int *flag, hipStream_t s) {
  int64_t total = nrows * ncols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) return;
  hipLaunchKernelGGL((nonfinite_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, X, ld, nrows, ncols, flag);
}
template void nonfinite_launch<double>(const double *, int64_t, int64_t, int, int *, hipStream_t);
template void nonfinite_launch<float>(const float *, int64_t, int64_t, int, int *, hipStream_t);

}  // namespace chfsi
