// Host-side launchers of the device kernels (internal interface of the library).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace chfsi {

// ---- Chebyshev step (hx.hip) ----------------------------------------------
// One Chebyshev step Y = s1 (Htilde - shift) X + s2 Xp, launched colour by colour
// (colours 0..7 in order; the first colour writes Y, later colours add).
template <typename T>
struct HxArgs {
  const T *X;          // input block, [n_dof x ldx]
  int64_t ldx;
  const T *Xp;         // previous block or nullptr (s2 ignored)
  int64_t ldp;
  T *Y;                // output block
  int64_t ldy;
  const T *K;          // padded cell stiffness [np x np]
  const int32_t *cmap; // [n_cells x n_loc]
  int n_loc, np, q, n_el;
  const int32_t *cells;  // cell ids sorted by colour
  const T *minv;       // M^-1/2 [n_dof]
  const T *V;          // potential [n_dof]
  int ncols;
  T s1, s2, shift;
  int variant;         // tile configuration: -1 built-in choice, 0 four-wave, 1 eight-wave
  int cpt = 1;         // cells per work-group (1, 2 or 4): the tile's columns split over that many cells
};
template <typename T>
int hx_cells_launch(const HxArgs<T> &a, int color_begin, int color_end, hipStream_t s);
// Columns per cell of one work-group of the cell kernel for padded cell size
// np, tile variant and cells per tile (-1 if not supported); the column
// tiles of the batched work list use it.
template <typename T>
int hx_tile_width(int np, int variant, int cpt);
// Degrees 8..12: row-group kernel, a.K stored [a.np][npr] (a.np = n_loc
// rounded up to 16, npr = hx_rows_padded(n_loc)), zero padded; -1 for
// arguments it does not support.
template <typename T>
int hx_rows_launch(const HxArgs<T> &a, int npr, int color_begin, int color_end, hipStream_t s);
int hx_rows_padded(int n_loc);
// Complex cell products on interleaved (re, im) columns: a.K is the
// [A ; B^T] operator (2 np x np) and a.ncols counts real columns (even).
int hx_cells_cplx_launch(const HxArgs<double> &a, int color_begin, int color_end, hipStream_t s);
// A group of nk k-points in one launch per colour: block k at X + k xstride
// (Y + k ystride, real elements), cell operator at a.K + k kstride, shift[k]
// on the potential term (a.Xp, a.s1, a.s2 and a.shift unused).
struct CplxKpts {
  int nk;
  int64_t xstride, ystride, kstride;
  const double *shifts;
};
int hx_cells_cplx_kpts_launch(const HxArgs<double> &a, const CplxKpts &g, int color_begin, int color_end,
                              hipStream_t s);

// One problem of a batched filter sweep (device-resident descriptor).
template <typename T>
struct BatchProblem {
  T *buf[3];           // the three rotating recursion buffers
  int64_t ld[3];
  const T *K;          // padded cell stiffness
  const int32_t *cmap;
  const T *minv, *V;
  const T *coef;       // [degree x 3]: s1, s2, shift per step
  const int32_t *cells;  // the problem's cells sorted by colour
  int n_loc, q, n_el, ncols;
};
// Launch one Chebyshev step for a list of work items (int4: x = problem, y =
// first cell in the problem's colour-sorted cell list, z = column tile, w =
// number of cells, at most cpt, all of one colour) whose problems share the
// padded cell size np, tile variant and cells per tile.
template <typename T>
int hx_cells_batch_launch(int np, int variant, int cpt, const BatchProblem<T> *probs, const int4 *work, int nwork,
                          int step, int cur, int prev, int out, hipStream_t s);
// BF16 cell products: FP32 X/Y/minv, K_ref as BF16 hi (and lo when split),
// padded to npb = round_up(n_loc, 32).
struct HxBf16Args {
  const float *X;
  int64_t ldx;
  const float *Xp;
  int64_t ldp;
  float *Y;
  int64_t ldy;
  const __bf16 *Kh, *Kl;
  const int32_t *cmap;
  int n_loc, npb, q, n_el;
  const int32_t *cells;
  const float *minv, *V;
  int ncols;
  float s1, s2, shift;
  int split;
  int cbw = 2;         // 16-column blocks per wave: 2 (64-column tiles) or 1 (32-column tiles)
};
int hx_cells_bf16_launch(const HxBf16Args &a, int color_begin, int color_end, hipStream_t s);
// One problem of a batched BF16 sweep: its three recursion buffers (FP32), the
// BF16 hi/lo cell matrix (npb x npb), maps and per-step coefficients.
struct BatchProblemBf16 {
  float *buf[3];
  int64_t ld[3];
  const __bf16 *Kh, *Kl;
  const int32_t *cmap, *cells;
  const float *minv, *V, *coef;
  int n_loc, q, n_el, ncols;
};
// work items (problem, cell position, 64-column tile, unused) of one padded
// size npb (32 .. 512) and one colour; -1 for an unsupported npb
int hx_cells_bf16_batch_launch(int npb, int split, const BatchProblemBf16 *probs, const int4 *work, int nwork,
                               int step, int cur, int prev, int out, hipStream_t s);
template <typename Tin, typename Tout>
void copy_cols_launch(const Tin *in, int64_t ldi, Tout *out, int64_t ldo, int64_t nrows, int ncols,
                      hipStream_t s);
template <typename T>
void nonfinite_launch(const T *X, int64_t ld, int64_t nrows, int ncols, int *flag, hipStream_t s);

// ---- tall-skinny products (dense.hip) ---------------------------------------
// G = A^T B over nrows rows, lower-triangular 128x128 tiles, split over rows;
// partial tiles go to `part` ([nsplit x ntiles x 128 x 128]) and are summed in
// a fixed order into G (n x n, row-major, lower triangle mirrored to upper).
// mixed: 64x64 diagonal blocks in FP64, the rest with FP32 inputs/products.
// nsplit is sized from the device's resident work-groups; gram_part_elems is
// the partial buffer for any gram launch on the current device, and
// gram_part_elems_slots the same for a given resident count (no device query).
int gram_nsplit(int64_t nrows, int n);
size_t gram_part_elems(int64_t nrows, int n);
size_t gram_part_elems_slots(int64_t nrows, int n, int slots);
void gram_launch(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrows, int n, double *part,
                 double *G, int mixed, hipStream_t s);
// As gram_launch with a partial buffer of part_elems doubles (0: sized by
// gram_part_elems): fewer row splits when it holds less; -1 when it cannot
// hold one split of every tile.
int gram_launch_capped(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrows, int n,
                       double *part, size_t part_elems, double *G, int mixed, hipStream_t s);
// As gram_launch, with the trailing block (rows and columns >= fr0, rounded
// down to a multiple of 64) in FP64 and everything else with FP32 inputs and
// products: the split projected Hamiltonian.
void gram_split_launch(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t nrows, int n, double *part,
                       double *G, int fr0, hipStream_t s);
// X[r, 0:n] <- X[r, 0:n] W for all rows, chunk by chunk through `scratch`
// (scratch_elems doubles, at least 128 x n; rmul_scratch_elems gives the size
// used by the library).  W: n x n row-major.  upper: W upper triangular (zero
// blocks skipped).  mixed (requires upper): the 64-wide diagonal blocks of W in
// FP64, the rest with FP32 inputs and products.  Returns -1 on bad arguments.
size_t rmul_scratch_elems(int64_t nrows, int n);
int rmul_launch(double *X, int64_t ld, int64_t nrows, int n, const double *W, int upper, int mixed,
                double *scratch, size_t scratch_elems, hipStream_t s);
// X[r, out_col0 : out_col0+nout] <- X[r, 0:n] W[0:n, 0:nout] (W row stride ldw),
// for all rows, chunk by chunk through `scratch` (as above); a partial
// rotation when nout < n.  upper/mixed as above (upper requires nout = ldw = n).
int rmul_cols_launch(double *X, int64_t ld, int64_t nrows, int n, const double *W, int64_t ldw, int nout,
                     int out_col0, int upper, int mixed, double *scratch, size_t scratch_elems, hipStream_t s);
// C[r, 0:nout] = X[r, 0:n] W[0:n, 0:nout] for all rows, out of place (C must
// not overlap X); one launch.  Returns -1 when the grid would not fit.
int rmul_out_launch(const double *X, int64_t ld, int64_t nrows, int n, const double *W, int64_t ldw, int nout,
                    double *C, int64_t ldc, hipStream_t s);
// rho[j] = 2 minv[j]^2 (sum_{i<ncols} X[j,i]^2 + sum_{k<nfr} w[k] Xfr[j,k]^2),
// j < nrows; w on the device.
void density_launch(const double *X, int64_t ld, int ncols, const double *Xfr, int64_t ldfr, int nfr,
                    const double *w, const double *minv, int64_t nrows, double *rho, hipStream_t s);
// resid[j] = || HX[:,j] - lam[j] X[:,j] ||_2 ; part: [nchunk x n]
int resid_nchunk(int64_t nrows);
void resid_launch(const double *X, int64_t ldx, const double *HX, int64_t ldh, const double *lam, int64_t nrows,
                  int n, double *part, double *resid, hipStream_t s);

// ---- small dense FP64 kernels (small.hip) ---------------------------------
// In-place blocked Cholesky of the lower triangle of S (n x n row-major):
// S + shift_rel*max(diag S)*I = L L^T; dinv receives the inverses of the 32x32
// diagonal blocks of L; *flag = first failing pivot + 1 (0 if every pivot
// d_j > 1e-14 * diag_j); diag0 [n] scratch; minratio[ceil(n/32)] = per-block
// minimum of d_j / diag_j.
void potrf_launch(double *S, int n, double *dinv, int *flag, double *diag0, double *minratio, double shift_rel,
                  hipStream_t s);
// W = L^-T (upper triangular, n x n row-major) from L and dinv; Z scratch n x n.
void trtri_t_launch(const double *L, const double *dinv, int n, double *Z, double *W, hipStream_t s);
// Symmetric eigensolver (cyclic Jacobi, round-robin pairs, one launch per round).
// A: n x n symmetric (row-major, full), destroyed; work: see jacobi_work_elems.
// On exit: evals ascending (device, n), Q (n x n row-major, columns = vectors).
size_t jacobi_work_elems(int n);
// Many independent eigenproblems at once: every round launch covers all
// problems still iterating, one host synchronisation per sweep checks them
// all.  Job k: A (destroyed), work (jacobi_work_elems(n)), evals/Q as above.
// table: device scratch of jacobi_table_bytes(njobs); norms: device and
// host_norms: host, jacobi_norms_elems(njobs) doubles each (jacobi_eigh:
// host_scratch of jacobi_norms_elems(1)).
struct JacobiJob {
  double *A;
  int n;
  double *work, *evals, *Q;
};
size_t jacobi_table_bytes(int njobs);
size_t jacobi_norms_elems(int njobs);
// Returns -1 on a HIP error, else the number of jobs whose off-diagonal norm
// had not met tol when max_sweeps sweeps were done (their evals/Q hold the
// last iterate); converged (may be null) receives 1/0 per job.
int jacobi_eigh_batch(const JacobiJob *jobs, int njobs, double tol, int max_sweeps, void *table, double *norms,
                      double *host_norms, hipStream_t s, int *sweeps_done, int *converged);
int jacobi_eigh(double *A, int n, double *work, double *evals, double *Q, double tol, int max_sweeps,
                double *host_scratch, hipStream_t s, int *sweeps_done);
// ---- complex (Hermitian) subspace steps on interleaved blocks (complex.hip)
// A complex n x N block X seen as the real n x 2N block R of its interleaved
// (re, im) columns.  G = R^T B (real 2N x 2N, lower triangle used) of two such
// blocks gives the Hermitian N x N matrix M = X^H Y through
//   Re M_jk = G[2j][2k] + G[2j+1][2k+1],  Im M_jk = G[2j][2k+1] - G[2j+1][2k]
// (j > k; the diagonal is real and the upper triangle follows by symmetry).
// herm_embed_launch writes E (2N x 2N real symmetric) = emb(M), the real form
// with 2 x 2 blocks [[Re, Im], [-Im, Re]], in which right-multiplication of R
// by emb(W) is the complex product X W.
void herm_embed_launch(const double *G, int n2, double *E, hipStream_t s);
// From the eigenvectors V (n2 x n2 row-major, column i = pair i, ascending
// values ev) of an embedded Hermitian matrix, where every eigenvalue appears
// twice, picks N = n2/2 complex eigenvectors: candidates in ascending order
// are orthogonalised (twice) against the kept w and J w (J the pair rotation,
// (Jw)_2j = -w_2j+1, (Jw)_2j+1 = w_2j) and kept when a tenth of their norm
// survives.  Q (n2 x n2) = [w_0, J w_0, w_1, J w_1, ...] is the embedding of
// the complex eigenvector matrix; evals [N] and lam2 [n2] (each value twice)
// receive the kept values; *status = number kept.  One work-group; n2 <= 4096.
void herm_select_launch(const double *V, const double *ev, int n2, double *Q, double *evals, double *lam2,
                        int *status, hipStream_t s);

// Zero the strictly upper triangle, helpers.
void fill_launch(double *X, int64_t n, double v, hipStream_t s);
void zero_int_launch(int *p, int n, hipStream_t s);

}  // namespace chfsi
