// Tall-skinny FP64 products of CholGS and Rayleigh-Ritz on MFMA.
//
//  * gram: G = A^T B, lower triangle only (Sec. 3.4 step 1, computing only the
//    lower-triangular part of the Hermitian overlap; Sec. 3.5 the projected
//    Hamiltonian the same way).  Mixed variant (eq. overlapmixedprec): FP64 on
//    the 64x64 diagonal blocks, FP32 inputs/products on the rest.
//  * rmul: X <- X W in place by row panels (Sec. 3.4 step 4, X L^-T; Sec. 3.5
//    subspace rotation X Q).  The paper's outer blocking over rows (B^d) keeps
//    only a panel of the output in extra memory: here a chunk of rows is
//    multiplied into a scratch panel and copied back.
//  * resid: column norms ||HX_j - lam_j X_j||.
//
// Launch shapes are sized from the device's resident work-group count (CUs x
// work-groups per CU at the kernel's occupancy), so that a grid ends just
// under a whole number of rounds: a grid of 4.04 rounds takes as long as one
// of 5.  Work-groups are dispatched to the 8 XCDs round-robin; the block index
// is remapped so that work-groups sharing operand rows (the tiles of one gram
// split, the column tiles of one rmul row tile) run on one XCD and share its
// L2.
#include "common.hpp"
#include "kernels.hpp"

#include <cmath>
#include <type_traits>

namespace chfsi {

static constexpr int GT = 128;  // gram output tile (4 waves x 64x64)

// Resident work-groups of `kern` (256 threads) on the current device.
template <typename K>
static int resident_slots(K kern) {
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 256, 0);
  return (cus > 0 ? cus : 1) * (per > 0 ? per : 1);
}

// Physical block index -> logical index such that the logical indices on one
// XCD (physical b = 8 i + x) are contiguous: XCD x holds [x*per + min(x, rem),
// ... + per + (x < rem)).
__device__ __forceinline__ int xcd_grouped_block() {
  const int g = (int)gridDim.x, b = (int)blockIdx.x;
  const int per = g >> 3, rem = g & 7, x = b & 7;
  return x * per + min(x, rem) + (b >> 3);
}

// lower-triangle tile enumeration t -> (ti, tj), ti >= tj
__device__ __forceinline__ void tri_tile(int t, int &ti, int &tj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// One (split, lower tile) work-group: partial G tile over rows [r0, r1).  The
// contraction runs over chunks of 16 rows: the chunk's 128 columns of A and
// of B are loaded into registers one chunk ahead (16-byte loads when the
// leading dimensions are even), written to the other half of a
// double-buffered LDS area after the chunk's MFMAs, and published by one
// barrier per chunk.  Wave (wi, wj) owns the 64 x 64 quarter (wi, wj); on a
// diagonal tile the strictly upper quarter is never read and is skipped.
// FP32 modes stage the chunk in LDS already rounded to FP32 (half the LDS
// bytes, so more resident work-groups).
// mode 0: every lower tile, FP64.  Mixed overlap: mode 1 computes every
// quarter except the 64 x 64 diagonal blocks with FP32 inputs and products,
// mode 2 (diagonal tiles only) the diagonal blocks in FP64.  Split projected
// Hamiltonian: mode 3 computes every quarter outside the trailing block
// (rows and columns >= fr0, fr0 a multiple of 64) with FP32 inputs and
// products, mode 4 the quarters inside it in FP64.
// Grid: nsplit x ngrid work-groups.  Modes 0, 1, 3: ngrid = ntl = all lower
// tiles.  Mode 2: ngrid = the diagonal tiles, part indexed by the full
// triangle (ntl tiles).  Mode 4: ngrid = ntl = the lower tiles of the trailing
// sub-triangle starting at tile row/column tf, part indexed within it.
template <int VEC, int MODE>
__global__ __launch_bounds__(256) void gram_kernel(const double *__restrict__ A, int64_t lda,
                                                   const double *__restrict__ B, int64_t ldb, int64_t nrows, int n,
                                                   int ngrid, int ntl, int tf, int64_t rows_per_split, int fr0,
                                                   double *__restrict__ part) {
  typedef double vec_t __attribute__((ext_vector_type(VEC)));
  typedef typename std::conditional<MODE == 1 || MODE == 3, float, double>::type CT;   // product type
  typedef typename acc4<CT>::type acc_t;
  typedef CT lds_vec_t __attribute__((ext_vector_type(VEC)));
  constexpr int KR = sizeof(CT) == 4 ? 32 : 16;   // rows per chunk (FP32 chunks: same LDS bytes)
  constexpr int PT = KR * GT / (256 * VEC);       // vectors per thread per operand
  // staged in the product type: FP32 modes round once, at the LDS store
  __shared__ __align__(16) CT As[2][KR][GT];
  __shared__ __align__(16) CT Bs[2][KR][GT];
  const int lid = xcd_grouped_block();
  const int split = lid / ngrid;
  int t = lid - split * ngrid;                    // part tile index
  int ti, tj;
  if (MODE == 2) {
    ti = tj = t;                                  // diagonal tile t
    t = ti * (ti + 1) / 2 + ti;
  } else {
    tri_tile(t, ti, tj);
    ti += tf;
    tj += tf;
  }
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wi = wave >> 1, wj = wave & 1;
  const int j = lane & 15, kq = lane >> 4;
  auto quarter_active = [&](int qi, int qj) {
    // strictly upper quarters and quarters wholly past the last column are never read
    const bool inside = ti * GT + qi * 64 < n && tj * GT + qj * 64 < n;
    const bool lower = !(ti == tj && qi < qj);
    const bool in_fr = ti * GT + qi * 64 >= fr0 && tj * GT + qj * 64 >= fr0;
    return inside && (MODE == 0 ? lower : MODE == 1 ? !(ti == tj && qi <= qj) : MODE == 2 ? qi == qj
                      : MODE == 3 ? lower && !in_fr : lower && in_fr);
  };
  if (!(quarter_active(0, 0) || quarter_active(1, 0) || quarter_active(0, 1) || quarter_active(1, 1)))
    return;                                        // whole work-group idle in this mode
  const bool active = quarter_active(wi, wj);
  const int64_t r0 = (int64_t)split * rows_per_split;
  int64_t r1 = r0 + rows_per_split;
  if (r1 > nrows) r1 = nrows;
  const int ib = ti * GT, jb = tj * GT;           // tile origin

  vec_t areg[PT], breg[PT];
  // slot v -> (row v / (GT/VEC), column vector v % (GT/VEC)); out-of-range
  // slots load a clamped in-bounds address and store zero
  auto load_chunk = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int v = tid + 256 * i;
      const int64_t row = min(k0 + v / (GT / VEC), r1 - 1);
      const int cv = (v % (GT / VEC)) * VEC;
      areg[i] = *reinterpret_cast<const vec_t *>(A + row * lda + min(ib + cv, n - VEC));
      breg[i] = *reinterpret_cast<const vec_t *>(B + row * ldb + min(jb + cv, n - VEC));
    }
  };
  auto store_chunk = [&](int buf, int64_t k0) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int v = tid + 256 * i;
      const int kr = v / (GT / VEC), cv = (v % (GT / VEC)) * VEC;
      const bool rok = k0 + kr < r1;
      lds_vec_t a, b;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        a[e] = (rok && ib + cv + e < n) ? (CT)areg[i][e] : (CT)0;
        b[e] = (rok && jb + cv + e < n) ? (CT)breg[i][e] : (CT)0;
      }
      *reinterpret_cast<lds_vec_t *>(&As[buf][kr][cv]) = a;
      *reinterpret_cast<lds_vec_t *>(&Bs[buf][kr][cv]) = b;
    }
  };

  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  const int64_t nk = (r1 - r0 + KR - 1) / KR;
  if (nk > 0) {
    load_chunk(r0);
    store_chunk(0, r0);
  }
  __syncthreads();
#pragma unroll 1
  for (int64_t kc = 0; kc < nk; ++kc) {
    const int buf = (int)(kc & 1);
    if (kc + 1 < nk) load_chunk(r0 + (kc + 1) * KR);
    if (active) {
#pragma unroll
      for (int ks = 0; ks < KR; ks += 4) {
        const int kk = ks + kq;
        CT av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = As[buf][kk][wi * 64 + a * 16 + j];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = Bs[buf][kk][wj * 64 + b * 16 + j];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = mfma16x4(av[a], bv[b], acc[a][b]);
      }
    }
    if (kc + 1 < nk) store_chunk(buf ^ 1, r0 + (kc + 1) * KR);
    __syncthreads();
  }
  if (!active) return;
  double *out = part + ((int64_t)split * ntl + t) * (GT * GT) + (wi * 64) * GT + wj * 64;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        out[(a * 16 + acc_row<CT>(kq, q)) * GT + b * 16 + j] = (double)acc[a][b][q];
      }
}

// G[i, j] = sum over splits of the partial tiles, for i >= j in the region
// [r0, n) x [r0, n) (tiles numbered within the sub-triangle from tile row tf),
// mirrored to the upper triangle.  skip0 >= 0: leave out the entries with both
// i and j >= skip0 (written by another reduction).
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double *__restrict__ part, int nsplit, int ntl,
                                                          int n, int tf, int r0, int skip0,
                                                          double *__restrict__ G) {
  const int m = n - r0;
  const int64_t total = (int64_t)m * m;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = r0 + (int)(idx / m), jj = r0 + (int)(idx - idx / m * m);
    if (jj > i || (skip0 >= 0 && jj >= skip0)) continue;
    const int ti = i / GT - tf, tj = jj / GT - tf;
    const int t = ti * (ti + 1) / 2 + tj;
    const double *p = part + (int64_t)t * (GT * GT) + (i % GT) * GT + (jj % GT);
    double s = 0;
    for (int sp = 0; sp < nsplit; ++sp) s += p[(int64_t)sp * ntl * (GT * GT)];
    G[(int64_t)i * n + jj] = s;
    G[(int64_t)jj * n + i] = s;
  }
}

static int gram_ntiles(int n) {
  int nt = (n + GT - 1) / GT;
  return nt * (nt + 1) / 2;
}

// Row splits for a launch of ntl tiles: the largest count whose grid fits in
// four rounds of `slots` resident work-groups, with at least 256 rows per split.
static int gram_nsplit_tiles(int64_t nrows, int ntl, int slots) {
  int64_t want = 4 * (int64_t)slots / ntl;
  const int64_t maxs = (nrows + 255) / 256;
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  return (int)want;
}

static int gram_slots() { return resident_slots(gram_kernel<2, 0>); }

int gram_nsplit(int64_t nrows, int n) { return gram_nsplit_tiles(nrows, gram_ntiles(n), gram_slots()); }

// Enough for a launch over the full triangle or over any trailing sub-triangle.
size_t gram_part_elems_slots(int64_t nrows, int n, int slots) {
  const int nt = (n + GT - 1) / GT;
  size_t best = 0;
  for (int m = 1; m <= nt; ++m) {
    const int ntl = m * (m + 1) / 2;
    const size_t e = (size_t)gram_nsplit_tiles(nrows, ntl, slots) * ntl;
    if (e > best) best = e;
  }
  return best * GT * GT;
}

size_t gram_part_elems(int64_t nrows, int n) { return gram_part_elems_slots(nrows, n, gram_slots()); }

static int64_t gram_rows_per_split(int64_t nrows, int nsplit) {
  int64_t rps = (nrows + nsplit - 1) / nsplit;
  return (rps + 15) / 16 * 16;
}

static void gram_reduce(const double *part, int nsplit, int ntl, int n, int tf, int r0, int skip0, double *G,
                        hipStream_t s) {
  const int64_t m = n - r0;
  int64_t blocks = (m * m + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) return;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, part, nsplit, ntl, n, tf, r0,
                     skip0, G);
}

static bool gram_v16(const double *A, int64_t lda, const double *B, int64_t ldb, int n) {
  return lda % 2 == 0 && ldb % 2 == 0 && n % 2 == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)B % 16) == 0;
}

template <int MODE>
static void gram_mode(bool v16, dim3 grid, const double *A, int64_t lda, const double *B, int64_t ldb,
                      int64_t nrows, int n, int ngrid, int ntl, int tf, int64_t rps, int fr0, double *part,
                      hipStream_t s) {
  if (v16)
    hipLaunchKernelGGL((gram_kernel<2, MODE>), grid, dim3(256), 0, s, A, lda, B, ldb, nrows, n, ngrid, ntl, tf, rps,
                       fr0, part);
  else
    hipLaunchKernelGGL((gram_kernel<1, MODE>), grid, dim3(256), 0, s, A, lda, B, ldb, nrows, n, ngrid, ntl, tf, rps,
                       fr0, part);
}

void gram_launch(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrows, int n, double *part,
                 double *G, int mixed, hipStream_t s) {
  gram_launch_capped(A, lda, B, ldb, nrows, n, part, 0, G, mixed, s);
}

int gram_launch_capped(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrows, int n,
                       double *part, size_t part_elems, double *G, int mixed, hipStream_t s) {
  const int ntiles = gram_ntiles(n);
  int nsplit = gram_nsplit_tiles(nrows, ntiles, gram_slots());
  if (part_elems > 0) {
    const size_t fit = part_elems / ((size_t)ntiles * GT * GT);
    if (fit < 1) return -1;
    if ((size_t)nsplit > fit) nsplit = (int)fit;
  }
  const int64_t rps = gram_rows_per_split(nrows, nsplit);
  const bool v16 = gram_v16(A, lda, B, ldb, n);
  const int nt = (n + GT - 1) / GT;
  const dim3 all((unsigned)(nsplit * ntiles)), diag((unsigned)(nsplit * nt));
  if (!mixed) {
    gram_mode<0>(v16, all, A, lda, B, ldb, nrows, n, ntiles, ntiles, 0, rps, 0, part, s);
  } else {
    gram_mode<1>(v16, all, A, lda, B, ldb, nrows, n, ntiles, ntiles, 0, rps, 0, part, s);
    gram_mode<2>(v16, diag, A, lda, B, ldb, nrows, n, nt, ntiles, 0, rps, 0, part, s);
  }
  gram_reduce(part, nsplit, ntiles, n, 0, 0, -1, G, s);
  return 0;
}

void gram_split_launch(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrows, int n, double *part,
                       double *G, int fr0, hipStream_t s) {
  fr0 = fr0 / 64 * 64;
  const bool v16 = gram_v16(A, lda, B, ldb, n);
  // the trailing block in FP64, on a grid over its own sub-triangle of tiles
  // (so that the few tiles it touches get every row split), reduced first
  const int nt = (n + GT - 1) / GT, tf = fr0 / GT, m = nt - tf;
  const int ntl4 = m * (m + 1) / 2;
  const int slots = gram_slots();
  const int nsplit4 = gram_nsplit_tiles(nrows, ntl4, slots);
  gram_mode<4>(v16, dim3((unsigned)(nsplit4 * ntl4)), A, lda, B, ldb, nrows, n, ntl4, ntl4, tf,
               gram_rows_per_split(nrows, nsplit4), fr0, part, s);
  gram_reduce(part, nsplit4, ntl4, n, tf, fr0, -1, G, s);
  if (fr0 == 0) return;
  // everything else with FP32 inputs and products; part is reused in order
  const int ntiles = gram_ntiles(n);
  const int nsplit = gram_nsplit_tiles(nrows, ntiles, slots);
  gram_mode<3>(v16, dim3((unsigned)(nsplit * ntiles)), A, lda, B, ldb, nrows, n, ntiles, ntiles, 0,
               gram_rows_per_split(nrows, nsplit), fr0, part, s);
  gram_reduce(part, nsplit, ntiles, n, 0, 0, fr0, G, s);
}

// ---------------------------------------------------------------------------
// Right multiplication X <- X W.  Rows are processed in chunks: an LDS-tiled
// MFMA GEMM writes C = X_chunk W into a scratch chunk, a coalesced copy puts
// it back (the paper's outer blocking over rows, which needs only a chunk of
// extra memory).  Work-group tile 128 x 128 (4 waves x 64 x 64); the
// contraction runs over chunks of 16: the X chunk (128 rows x 16, stored
// transposed so a fragment read is 16 consecutive words) and the W chunk
// (16 x 128) are loaded into registers one chunk ahead (16-byte loads when
// the leading dimensions are even), written to the other half of a
// double-buffered LDS area after the chunk's MFMAs, and published by one
// barrier per chunk.  upper: W upper triangular, so output column tile
// [n0, n0+128) only needs k < n0 + 128.  mixed (upper only): k in the
// 64-wide diagonal block of a wave's columns in FP64, smaller k in FP32.
// ---------------------------------------------------------------------------
static constexpr int MT = 128, NTL = 128, KC = 16;

// C[r, 0:nout] = X[row0 + r, 0:n] W[0:n, 0:nout] (W row stride ldw)
template <bool MIXED, int VEC>
__global__ __launch_bounds__(256) void rmul_gemm_kernel(const double *__restrict__ X, int64_t ld, int64_t row0,
                                                        int64_t nrows, int n, const double *__restrict__ W,
                                                        int64_t ldw, int nout, int upper, double *__restrict__ C,
                                                        int64_t ldc) {
  typedef double vec_t __attribute__((ext_vector_type(VEC)));
  constexpr int APT = KC * MT / (256 * VEC);     // X vectors per thread per chunk
  constexpr int WPT = KC * NTL / (256 * VEC);    // W vectors per thread per chunk
  __shared__ __align__(16) double As[2][KC][MT];   // As[k][row]
  __shared__ __align__(16) double Ws[2][KC][NTL];  // Ws[k][col]
  const int nt = (nout + NTL - 1) / NTL;
  const int lid = xcd_grouped_block();
  const int mt = lid / nt;
  const int ntile = lid - mt * nt;
  const int64_t r0 = row0 + (int64_t)mt * MT;    // first X row of this tile
  const int64_t rlast = row0 + nrows - 1;         // last valid row
  const int n0 = ntile * NTL;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wi = wave >> 1, wj = wave & 1;
  const int j = lane & 15, kq = lane >> 4;
  const int kend = upper ? min(n, n0 + NTL) : n;
  const int c0 = n0 + wj * 64;                   // first column of this wave
  const bool live = c0 < nout;                   // a wave wholly past nout skips its MFMAs
  const int kdiag = MIXED ? (c0 / 64) * 64 : 0;  // mixed: k >= kdiag is the FP64 diagonal block

  // staging slots: X vector v -> (row v % MT, k-vector v / MT); W vector v ->
  // (k-row v / (NTL/VEC), column vector v % (NTL/VEC)).  Out-of-range slots
  // load a clamped in-bounds address and store zero.
  vec_t areg[APT], wreg[WPT];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      const int v = tid + 256 * i;
      const int64_t row = min(r0 + v % MT, rlast);
      const int k = min(k0 + (v / MT) * VEC, n - VEC);
      areg[i] = *reinterpret_cast<const vec_t *>(X + row * ld + k);
    }
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int v = tid + 256 * i;
      const int k = min(k0 + v / (NTL / VEC), n - 1);
      const int col = min(n0 + (v % (NTL / VEC)) * VEC, nout - VEC);
      wreg[i] = *reinterpret_cast<const vec_t *>(W + (int64_t)k * ldw + col);
    }
  };
  auto store_chunk = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      const int v = tid + 256 * i;
      const int r = v % MT, kv = (v / MT) * VEC;
      const bool rok = r0 + r <= rlast;
#pragma unroll
      for (int e = 0; e < VEC; ++e) As[buf][kv + e][r] = (rok && k0 + kv + e < n) ? areg[i][e] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int v = tid + 256 * i;
      const int kr = v / (NTL / VEC), cv = (v % (NTL / VEC)) * VEC;
      vec_t w = wreg[i];
      const bool kok = k0 + kr < kend;
#pragma unroll
      for (int e = 0; e < VEC; ++e) w[e] = (kok && n0 + cv + e < nout) ? w[e] : 0.0;
      *reinterpret_cast<vec_t *>(&Ws[buf][kr][cv]) = w;
    }
  };

  // one pipeline step: prefetch chunk kc + 1, multiply chunk kc, publish
  // chunk kc + 1.  F32: FP32 inputs and products into acc32.
  const int nk = (kend + KC - 1) / KC;
  auto step = [&](int kc, auto f32, auto &accs) {
    const int buf = kc & 1;
    if (kc + 1 < nk) load_chunk((kc + 1) * KC);
#pragma unroll
    for (int ks = 0; ks < KC && live; ks += 4) {
      const int kk = ks + kq;
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[buf][kk][wi * 64 + a * 16 + j];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Ws[buf][kk][wj * 64 + b * 16 + j];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if constexpr (decltype(f32)::value)
            accs[a][b] = mfma16x4((float)av[a], (float)bv[b], accs[a][b]);
          else
            accs[a][b] = mfma16x4(av[a], bv[b], accs[a][b]);
        }
    }
    if (kc + 1 < nk) store_chunk(buf ^ 1, (kc + 1) * KC);
    __syncthreads();
  };

  load_chunk(0);
  store_chunk(0, 0);
  __syncthreads();
  v4d acc[4][4];
  int kc = 0;
  if constexpr (MIXED) {
    // chunks left of the wave's diagonal block in FP32 (kdiag is a multiple
    // of 64, so chunks never straddle it), then the FP64 accumulators start
    // from the converted FP32 sums
    const int nk32 = min(kdiag / KC, nk);
    v4f acc32[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc32[a][b] = v4f{0, 0, 0, 0};
#pragma unroll 1
    for (; kc < nk32; ++kc) step(kc, std::true_type{}, acc32);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = f32acc_to_f64_layout(acc32[a][b], lane);
  } else {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0, 0, 0, 0};
  }
#pragma unroll 1
  for (; kc < nk; ++kc) step(kc, std::false_type{}, acc);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t rr = (int64_t)mt * MT + wi * 64 + a * 16 + acc_row<double>(kq, q);  // chunk-local row
        const int col = c0 + b * 16 + j;
        if (rr < nrows && col < nout) C[rr * ldc + col] = acc[a][b][q];
      }
}

__global__ __launch_bounds__(256) void copy_back_kernel(const double *__restrict__ C, int64_t ldc, double *X,
                                                        int64_t ld, int64_t row0, int64_t nrows, int n,
                                                        int col0) {
  const int64_t total = nrows * (int64_t)n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / n;
    const int c = (int)(t - r * n);
    X[(row0 + r) * ld + col0 + c] = C[r * ldc + c];
  }
}

size_t rmul_scratch_elems(int64_t nrows, int n) {
  // at most 1 GiB, and no more than the whole product needs
  const int64_t cap = (int64_t)1 << 27;
  const int64_t all = (nrows + MT - 1) / MT * MT * (int64_t)(n > 0 ? n : 1);
  int64_t e = all < cap ? all : cap;
  if (e < (int64_t)MT * n) e = (int64_t)MT * n;
  return (size_t)e;
}

int rmul_cols_launch(double *X, int64_t ld, int64_t nrows, int n, const double *W, int64_t ldw, int nout,
                     int out_col0, int upper, int mixed, double *scratch, size_t scratch_elems, hipStream_t s) {
  if (mixed && !upper) return -1;
  if (upper && (nout != n || ldw != n)) return -1;
  if (n <= 0 || nout <= 0 || nrows <= 0) return 0;
  if (scratch_elems < (size_t)MT * nout) return -1;
  const int nt = (nout + NTL - 1) / NTL;
  // row tiles per launch: as many as the scratch panel holds, rounded down to
  // whole rounds of resident work-groups when there is more than one round
  const int64_t mts_all = (nrows + MT - 1) / MT;
  int64_t mts_chunk = (int64_t)(scratch_elems / nout) / MT;
  if (mts_chunk < mts_all) {
    const int64_t slots = mixed ? resident_slots(rmul_gemm_kernel<true, 2>) : resident_slots(rmul_gemm_kernel<false, 2>);
    const int64_t rounds = mts_chunk * nt / slots;
    if (rounds >= 1) mts_chunk = rounds * slots / nt;
  } else {
    mts_chunk = mts_all;
  }
  if (mts_chunk < 1) mts_chunk = 1;
  const int64_t chunk = mts_chunk * MT;
  // 16-byte operand loads need even leading dimensions and 16-byte aligned bases
  const bool v16 = ld % 2 == 0 && n % 2 == 0 && ldw % 2 == 0 && nout % 2 == 0 && ((uintptr_t)X % 16) == 0 &&
                   ((uintptr_t)W % 16) == 0;
  for (int64_t r = 0; r < nrows; r += chunk) {
    const int64_t rows = (nrows - r < chunk) ? nrows - r : chunk;
    const int64_t mts = (rows + MT - 1) / MT;
    const dim3 grid((unsigned)(mts * nt)), block(256);
    const int64_t ldc = nout;
    if (mixed) {
      if (v16) hipLaunchKernelGGL((rmul_gemm_kernel<true, 2>), grid, block, 0, s, X, ld, r, rows, n, W, ldw, nout, upper, scratch, ldc);
      else hipLaunchKernelGGL((rmul_gemm_kernel<true, 1>), grid, block, 0, s, X, ld, r, rows, n, W, ldw, nout, upper, scratch, ldc);
    } else {
      if (v16) hipLaunchKernelGGL((rmul_gemm_kernel<false, 2>), grid, block, 0, s, X, ld, r, rows, n, W, ldw, nout, upper, scratch, ldc);
      else hipLaunchKernelGGL((rmul_gemm_kernel<false, 1>), grid, block, 0, s, X, ld, r, rows, n, W, ldw, nout, upper, scratch, ldc);
    }
    int64_t total = rows * nout;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(copy_back_kernel, dim3((unsigned)blocks), dim3(256), 0, s, scratch, ldc, X, ld, r, rows, nout,
                       out_col0);
  }
  return 0;
}

int rmul_launch(double *X, int64_t ld, int64_t nrows, int n, const double *W, int upper, int mixed,
                double *scratch, size_t scratch_elems, hipStream_t s) {
  return rmul_cols_launch(X, ld, nrows, n, W, n, n, 0, upper, mixed, scratch, scratch_elems, s);
}

int rmul_out_launch(const double *X, int64_t ld, int64_t nrows, int n, const double *W, int64_t ldw, int nout,
                    double *C, int64_t ldc, hipStream_t s) {
  if (n <= 0 || nout <= 0 || nrows <= 0) return 0;
  const bool v16 = ld % 2 == 0 && n % 2 == 0 && ldw % 2 == 0 && nout % 2 == 0 && ((uintptr_t)X % 16) == 0 &&
                   ((uintptr_t)W % 16) == 0;
  const int nt = (nout + NTL - 1) / NTL;
  const int64_t mts = (nrows + MT - 1) / MT;
  if (mts * nt > INT32_MAX) return -1;
  const dim3 grid((unsigned)(mts * nt)), block(256);
  if (v16) hipLaunchKernelGGL((rmul_gemm_kernel<false, 2>), grid, block, 0, s, X, ld, 0, nrows, n, W, ldw, nout, 0, C, ldc);
  else hipLaunchKernelGGL((rmul_gemm_kernel<false, 1>), grid, block, 0, s, X, ld, 0, nrows, n, W, ldw, nout, 0, C, ldc);
  return 0;
}

// ---------------------------------------------------------------------------
// Nodal electron density (Alg. 5, eq. elecDensSP with the collocated GLL
// rule): rho_j = 2 minv_j^2 (sum_i X[j,i]^2 + sum_k w_k Xfr[j,k]^2), w_k =
// f(eps_k, mu) - 1.  One wave per DoF row (a row is contiguous in the
// DoF-major layout, so a wave's loads are coalesced), lanes over columns with
// 16-byte loads where the layout allows, a fixed shuffle tree for the sum.
// HBM-bound: 8 (ncols + nfr) + 16 bytes per DoF.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <bool V2, bool F2>
__global__ __launch_bounds__(256) void density_kernel(const double *__restrict__ X, int64_t ld, int ncols,
                                                      const double *__restrict__ Xfr, int64_t ldfr, int nfr,
                                                      const double *__restrict__ w, const double *__restrict__ minv,
                                                      int64_t nrows, double *__restrict__ rho) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t row = wid; row < nrows; row += stride) {
    const double *xr = X + row * ld;
    double s0 = 0, s1 = 0;
    if (V2) {
      // two 16-byte loads per lane per step (a deeper unroll measured slower)
      int c = 2 * lane;
      for (; c + 128 < ncols; c += 256) {
        const d2 a = *reinterpret_cast<const d2 *>(xr + c);
        const d2 b = *reinterpret_cast<const d2 *>(xr + c + 128);
        s0 += a[0] * a[0] + a[1] * a[1];
        s1 += b[0] * b[0] + b[1] * b[1];
      }
      if (c < ncols) {
        const d2 a = *reinterpret_cast<const d2 *>(xr + c);
        s0 += a[0] * a[0] + a[1] * a[1];
      }
    } else {
      for (int c = lane; c < ncols; c += 64) {
        const double v = xr[c];
        s0 += v * v;
      }
    }
    const double *fr = Xfr + row * ldfr;
    if (F2) {
      for (int c = 2 * lane; c < nfr; c += 128) {
        const d2 v = *reinterpret_cast<const d2 *>(fr + c);
        const d2 wk = *reinterpret_cast<const d2 *>(w + c);
        s1 += wk[0] * (v[0] * v[0]) + wk[1] * (v[1] * v[1]);
      }
    } else {
      for (int c = lane; c < nfr; c += 64) {
        const double v = fr[c];
        s1 += w[c] * (v * v);
      }
    }
    const double tot = wave_sum(s0 + s1);
    if (lane == 0) {
      const double m = minv[row];
      rho[row] = 2.0 * (m * m) * tot;
    }
  }
}

void density_launch(const double *X, int64_t ld, int ncols, const double *Xfr, int64_t ldfr, int nfr,
                    const double *w, const double *minv, int64_t nrows, double *rho, hipStream_t s) {
  if (nrows <= 0) return;
  int64_t blocks = (nrows + 3) / 4;
  if (blocks > 8192) blocks = 8192;
  const dim3 g((unsigned)blocks), b(256);
  const bool v2 = ld % 2 == 0 && ncols % 2 == 0 && ((uintptr_t)X % 16) == 0;
  const bool f2 = nfr > 0 && ldfr % 2 == 0 && nfr % 2 == 0 && ((uintptr_t)Xfr % 16) == 0 && ((uintptr_t)w % 16) == 0;
  if (v2 && f2) hipLaunchKernelGGL((density_kernel<true, true>), g, b, 0, s, X, ld, ncols, Xfr, ldfr, nfr, w, minv, nrows, rho);
  else if (v2) hipLaunchKernelGGL((density_kernel<true, false>), g, b, 0, s, X, ld, ncols, Xfr, ldfr, nfr, w, minv, nrows, rho);
  else if (f2) hipLaunchKernelGGL((density_kernel<false, true>), g, b, 0, s, X, ld, ncols, Xfr, ldfr, nfr, w, minv, nrows, rho);
  else hipLaunchKernelGGL((density_kernel<false, false>), g, b, 0, s, X, ld, ncols, Xfr, ldfr, nfr, w, minv, nrows, rho);
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
