// Chebyshev-step kernels: Y = s1 (Htilde - shift) X + s2 Xprev with
// Htilde X = M^-1/2 (sum_e P_e^T K_e P_e) M^-1/2 X + V .* X.
//
// Paper, Sec. 3.3 (practical implementation of Chebyshev filtering): store the
// cell Hamiltonian, extract the cell wavefunction matrices from the DoF-major
// global block, multiply, assemble.  On a uniform mesh every cell carries the
// same stiffness K_ref, so the cell products form one dense contraction
// K_ref [n_loc x n_loc] x X_e [n_loc x ncols] per cell, done here on MFMA.
// Under GLL quadrature the potential part is diagonal and is applied in the
// element-wise pass (hx_diag), which also initialises Y.
//
// Assembly is atomic-free: cells are launched colour by colour (8 colours,
// (ex&1)+2(ey&1)+4(ez&1)); cells of one colour share no DoF, so each output
// row is read-modified-written by exactly one work-group per launch.
#include "common.hpp"
#include "kernels.hpp"

namespace chfsi {

// ---------------------------------------------------------------------------
// Element-wise pass: Y[i,j] = s1 (V[i] - shift) X[i,j] + s2 Xprev[i,j]
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void hx_diag_kernel(const T *__restrict__ X, int64_t ldx,
                                                      const T *__restrict__ Xp, int64_t ldp,
                                                      T *__restrict__ Y, int64_t ldy,
                                                      const T *__restrict__ V, int64_t n_dof, int ncols,
                                                      T s1, T s2, T shift) {
  const int64_t total = n_dof * (int64_t)ncols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = t / ncols;
    int j = (int)(t - i * ncols);
    T y = s1 * (V[i] - shift) * X[i * ldx + j];
    if (Xp) y += s2 * Xp[i * ldp + j];
    Y[i * ldy + j] = y;
  }
}

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

template <typename T, int NP>
__global__ __launch_bounds__(256) void hx_cells_kernel(const T *__restrict__ X, int64_t ldx,
                                                       T *__restrict__ Y, int64_t ldy,
                                                       const T *__restrict__ K,
                                                       const int32_t *__restrict__ cmap, int n_loc,
                                                       const int32_t *__restrict__ cells,
                                                       const T *__restrict__ minv, int ncols,
                                                       int ntiles, T s1) {
  typedef typename acc4<T>::type acc_t;
  constexpr int RB = CellTile<T, NP>::RB;
  constexpr int RBP = CellTile<T, NP>::RBP;
  __shared__ int32_t dof_s[NP];
  __shared__ T mi_s[NP];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cell_slot = blockIdx.x / ntiles;
  const int tile = blockIdx.x - cell_slot * ntiles;
  const int e = cells[cell_slot];
  for (int r = threadIdx.x; r < NP; r += blockDim.x) {
    int d = r < n_loc ? cmap[(int64_t)e * n_loc + r] : -1;
    dof_s[r] = d < 0 ? 0 : d;              // clamped: row 0 is always readable
    mi_s[r] = d < 0 ? T(0) : minv[d];      // zero weight removes Dirichlet / padding rows
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
#pragma unroll
      for (int r = 0; r < RBP; ++r) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = (rb0 + r) * 16 + acc_row<T>(kq, q);
          if (row < n_loc) {
            const T w = mi_s[row];
            if (w != T(0)) {
              T *yp = Y + (int64_t)dof_s[row] * ldy + col;
              *yp += s1 * w * acc[r][q];
            }
          }
        }
      }
    }
  }
}

template <typename T, int NP>
static void launch_cells(const HxArgs<T> &a, int color_begin, int color_end, hipStream_t s) {
  int ntiles = (a.ncols + 63) / 64;
  int ncell = color_end - color_begin;
  if (ncell <= 0 || ntiles <= 0) return;
  dim3 grid((unsigned)(ncell * ntiles)), block(256);
  hipLaunchKernelGGL((hx_cells_kernel<T, NP>), grid, block, 0, s, a.X, a.ldx, a.Y, a.ldy, a.K, a.cmap,
                     a.n_loc, a.cells + color_begin, a.minv, a.ncols, ntiles, a.s1);
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

template <typename T>
void hx_diag_launch(const T *X, int64_t ldx, const T *Xp, int64_t ldp, T *Y, int64_t ldy, const T *V,
                    int64_t n_dof, int ncols, T s1, T s2, T shift, hipStream_t s) {
  int64_t total = n_dof * ncols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((hx_diag_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, X, ldx, Xp, ldp, Y, ldy, V,
                     n_dof, ncols, s1, s2, shift);
}

template int hx_cells_launch<double>(const HxArgs<double> &, int, int, hipStream_t);
template int hx_cells_launch<float>(const HxArgs<float> &, int, int, hipStream_t);
template void hx_diag_launch<double>(const double *, int64_t, const double *, int64_t, double *, int64_t,
                                     const double *, int64_t, int, double, double, double, hipStream_t);
template void hx_diag_launch<float>(const float *, int64_t, const float *, int64_t, float *, int64_t,
                                    const float *, int64_t, int, float, float, float, hipStream_t);

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
