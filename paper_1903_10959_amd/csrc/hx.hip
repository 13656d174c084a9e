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
// columns [n0, n0+16) with n0 = 64*tile + 16*w and all NP/16 output row blocks.
// B operand: gathered, M^-1/2-scaled X rows of the cell (direct from global,
// each row segment 16 contiguous values).  A operand: K_ref (symmetric, padded
// to NP with zeros) read row-wise, so A[i][k] = K[k][i] is contiguous in i.
// Epilogue: Y[dof, col] += s1 * minv[dof] * acc.
// ---------------------------------------------------------------------------
template <typename T, int NP>
__global__ __launch_bounds__(256) void hx_cells_kernel(const T *__restrict__ X, int64_t ldx,
                                                       T *__restrict__ Y, int64_t ldy,
                                                       const T *__restrict__ K,
                                                       const int32_t *__restrict__ cmap, int n_loc,
                                                       const int32_t *__restrict__ cells,
                                                       const T *__restrict__ minv, int ncols,
                                                       int ntiles, T s1) {
  typedef typename acc4<T>::type acc_t;
  constexpr int RB = NP / 16;  // output row blocks
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cell_slot = blockIdx.x / ntiles;
  const int tile = blockIdx.x - cell_slot * ntiles;
  const int e = cells[cell_slot];
  const int j = lane & 15, kq = lane >> 4;
  const int col = tile * 64 + wave * 16 + j;
  const bool col_ok = col < ncols;
  const int32_t *__restrict__ cm = cmap + (int64_t)e * n_loc;

  // FP64 with NP = 512 would need 256 accumulator registers: two passes of 16 row blocks
  constexpr int RBP = (sizeof(T) == 8 && RB > 22) ? RB / 2 : RB;
  auto load_b = [&](int k) -> T {
    int row = 4 * k + kq;
    int d = row < n_loc ? cm[row] : -1;
    return (d >= 0 && col_ok) ? X[(int64_t)d * ldx + col] * minv[d] : T(0);
  };

  for (int rb0 = 0; rb0 < RB; rb0 += RBP) {
    acc_t acc[RBP];
#pragma unroll
    for (int r = 0; r < RBP; ++r) acc[r] = acc_t{0, 0, 0, 0};

    // software pipeline: operands of step k+1 are loaded while step k issues
    T b_cur = load_b(0);
    T a_cur[RBP];
#pragma unroll
    for (int r = 0; r < RBP; ++r) a_cur[r] = K[(int64_t)kq * NP + (rb0 + r) * 16 + j];

    for (int k = 0; k < NP / 4; ++k) {
      T b_nxt = T(0);
      T a_nxt[RBP];
#pragma unroll
      for (int r = 0; r < RBP; ++r) a_nxt[r] = T(0);
      if (k + 1 < NP / 4) {
        b_nxt = load_b(k + 1);
#pragma unroll
        for (int r = 0; r < RBP; ++r) a_nxt[r] = K[(int64_t)(4 * (k + 1) + kq) * NP + (rb0 + r) * 16 + j];
      }
#pragma unroll
      for (int r = 0; r < RBP; ++r) acc[r] = mfma16x4(a_cur[r], b_cur, acc[r]);
      b_cur = b_nxt;
#pragma unroll
      for (int r = 0; r < RBP; ++r) a_cur[r] = a_nxt[r];
    }

    if (col_ok) {
#pragma unroll
      for (int r = 0; r < RBP; ++r) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int row = (rb0 + r) * 16 + acc_row<T>(kq, q);
          if (row < n_loc) {
            int d = cm[row];
            if (d >= 0) {
              T *yp = Y + (int64_t)d * ldy + col;
              *yp += s1 * minv[d] * acc[r][q];
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
