/*
 * chfsi.h -- C ABI of the MI355X (gfx950) Chebyshev-filtered subspace
 * iteration library for the spectral finite-element Kohn-Sham operator.
 *
 * The operator is the standard form of the discrete eigenproblem
 * H psi = eps M psi (Sec. 2.4, eq. hep):
 *
 *     Htilde = M^-1/2 H M^-1/2,  H = K + diag(M V),
 *
 * on a uniform mesh of n_el^3 hexahedral cells of [0,L]^3 with C0 Lagrange
 * elements of degree p on Gauss-Lobatto-Legendre nodes, homogeneous Dirichlet
 * boundary (boundary nodes carry no unknown).  K is the stiffness of
 * -1/2 Laplacian (eq. discreteHam); GLL quadrature makes M diagonal, so
 * Htilde X = M^-1/2 (sum_e P_e^T K_e P_e) M^-1/2 X + V .* X, applied cell by
 * cell (Sec. 3.3, practical implementation of Chebyshev filtering).
 *
 * Conventions used by every call:
 *  - Return value: 0 = OK, < 0 = error (CHFSI_ERR_*), > 0 = warning.  No C++
 *    exception crosses this interface; chfsi_last_error() gives a message.
 *  - Blocks of vectors X are FP64, DoF-major ("for each degree of freedom the
 *    values of all vectors are stored contiguously", Sec. 3.3): element
 *    (dof i, column j) is X[i*ld + j], ld >= ncols.  All such pointers are
 *    DEVICE pointers owned by the caller; the library never frees them.
 *  - Numbering: interior node (I,J,K), 1 <= I,J,K <= n, n = n_el*p - 1, is
 *    dof (I-1) + n(J-1) + n^2(K-1); cell e = ex + n_el*ey + n_el^2*ez; local
 *    node l = a + (p+1)b + (p+1)^2 c with I = ex*p + a.
 *  - Streams: all device work is enqueued on the stream given at create time
 *    (borrowed, not owned).  Calls that return host data synchronise it.
 *  - Threads: one context is used by one host thread at a time.  Separate
 *    contexts on separate streams may run concurrently.
 *  - Units: Hartree and bohr.
 */
#ifndef CHFSI_H
#define CHFSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chfsi_ctx chfsi_ctx;   /* opaque; owned by the library */

/* Arithmetic of the filter's cell products.  FP64 = the paper's precision.
 * FP32: recursion state and products in FP32.  BF16: products with BF16
 * inputs and FP32 accumulation, recursion state FP32.  BF16X3: BF16 hi/lo
 * split of both operands, three products accumulated in FP32. */
typedef enum {
    CHFSI_FP64 = 0,
    CHFSI_FP32 = 1,
    CHFSI_BF16 = 2,
    CHFSI_BF16X3 = 3
} chfsi_prec;

enum {
    CHFSI_OK = 0,
    CHFSI_ERR_ARG = -1,        /* invalid argument (size, pointer, range)           */
    CHFSI_ERR_STATE = -2,      /* call order: mesh/potential not set                */
    CHFSI_ERR_OOM = -3,        /* device allocation failed                          */
    CHFSI_ERR_HIP = -4,        /* a HIP runtime call failed                         */
    CHFSI_ERR_NOT_SPD = -5,    /* Cholesky met a non-positive pivot (rank deficient) */
    CHFSI_ERR_NONFINITE = -6,  /* NaN/Inf produced (e.g. b below lambda_max)        */
    CHFSI_WARN_NOT_CONVERGED = 1
};

/* ---- lifetime ---------------------------------------------------------- */

/* Create a context on HIP device `device`; `hip_stream` (a hipStream_t, may be
 * NULL = the null stream) is borrowed for all later work.  device = -1 creates
 * a host-only context: set_mesh/set_potential build the host tables and the
 * bound, the get_* calls work, every device call returns CHFSI_ERR_STATE. */
int chfsi_create(chfsi_ctx **out, int device, void *hip_stream);
/* Free everything the context allocated (device buffers, host tables). */
int chfsi_destroy(chfsi_ctx *ctx);

/* ---- setMesh (Sec. 2.4 eq. fem, Sec. 3.1 mesh; uniform cubes only) ------
 * Build the GLL rule of degree p (1..12; CHFSI_ERR_ARG otherwise), the
 * reference cell stiffness
 * 1/2 (h/2)[K1 (x) W (x) W + W (x) K1 (x) W + W (x) W (x) K1] (h = L/n_el,
 * K1 = D^T W D, W = diag of GLL weights), the cell->dof map, the 8-colour
 * cell colouring (ex&1)+2(ey&1)+4(ez&1) and the diagonal mass M (GLL rule),
 * and upload them.  Resets any potential set before.  Requires n_el*p >= 2.
 * Degrees 8..12 (n_loc = 729..2197) run the FP64/FP32 cell products in groups
 * of 224 output rows per work-group; the BF16 products, the complex
 * k-point operator and the batch session need p <= 7 (CHFSI_ERR_ARG). */
int chfsi_set_mesh(chfsi_ctx *ctx, double L, int n_el, int p);
int chfsi_get_sizes(const chfsi_ctx *ctx, int64_t *n_dof, int64_t *n_cells, int *n_loc);
/* Host copies of the tables built by set_mesh (caller-owned host buffers). */
int chfsi_get_cell_dof_map(const chfsi_ctx *ctx, int32_t *host_out);  /* [n_cells*n_loc], -1 = Dirichlet */
int chfsi_get_cell_colors(const chfsi_ctx *ctx, uint8_t *host_out);   /* [n_cells] */
int chfsi_get_dof_coords(const chfsi_ctx *ctx, double *host_xyz);     /* [3*n_dof], x,y,z per dof */
int chfsi_get_mass(const chfsi_ctx *ctx, double *host_m);             /* [n_dof] diagonal of M */
int chfsi_get_cell_matrix(const chfsi_ctx *ctx, double *host_k);      /* [n_loc*n_loc] cell stiffness */

/* ---- setPotential (Sec. 2.4 eq. discreteHam, GLL quadrature) -----------
 * Nodal V (Ha) at the n_dof interior nodes, host (v_on_device = 0) or device
 * pointer; copied.  Also sets the filter's upper bound
 * b = 3 lambda_max(A_1D) + max V >= lambda_max(Htilde) (Weyl; A_1D is the
 * assembled 1D operator whose Kronecker sum is the kinetic part). */
int chfsi_set_potential(chfsi_ctx *ctx, const double *v, int64_t n_dof, int v_on_device);
int chfsi_get_upper_bound(const chfsi_ctx *ctx, double *b);

/* ---- Htilde X (Sec. 3.3: cell-level products, assembled) -----------------
 * Y = Htilde X for ncols columns.  X, Y: device, [n_dof x ld], must not alias.
 * prec selects the cell-product arithmetic (X, Y stay FP64). */
int chfsi_apply(chfsi_ctx *ctx, const double *X, double *Y, int64_t ld, int ncols, chfsi_prec prec);

/* One recursion step (eq. chebFilter, normalised form):
 * Y = s1 (Htilde - shift) X + s2 Xprev   (Xprev may be NULL when s2 == 0).
 * All device FP64 [n_dof x ld]; Y must not alias X or Xprev. */
int chfsi_cheb_step(chfsi_ctx *ctx, const double *X, const double *Xprev, double *Y,
                    int64_t ld, int ncols, double s1, double s2, double shift);

/* ---- chebyshevFilter (Sec. 3.3 eq. chebFilter) ----------------------------
 * In place: X <- T_m(Hbar) X / T_m(xi0), Hbar = (Htilde - c)/e,
 * c = (a+b)/2, e = (b-a)/2, xi0 = (a0-c)/e, requires a0 < a < b.
 * Vectors are filtered in blocks of block_width columns (0 = library default)
 * with three rotating buffers per block.  Returns CHFSI_ERR_NONFINITE if the
 * result holds NaN/Inf. */
int chfsi_chebyshev_filter(chfsi_ctx *ctx, double *X, int64_t ld, int ncols, int degree,
                           double a, double b, double a0, chfsi_prec prec, int block_width);

/* ---- orthonormalize (Sec. 3.4 Alg. 3, CholGS) ----------------------------
 * In place: S = X^T X, S = L L^T, L^-1, X <- X L^-T, so X^T X = I on return.
 * mixed = 1: the paper's mixed-precision split (eq. overlapmixedprec): FP64
 * diagonal blocks of S and of L^-T, FP32 off-diagonal blocks.
 * CHFSI_ERR_NOT_SPD if S is not numerically positive definite (X unchanged). */
int chfsi_orthonormalize(chfsi_ctx *ctx, double *X, int64_t ld, int ncols, int mixed);

/* ---- orthonormalize without allocating ----------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * CholGS as chfsi_orthonormalize (same kernels, same arguments, same errors,
 * X unchanged on CHFSI_ERR_NOT_SPD), with every workspace taken from one
 * static device array of CHFSI_NOALLOC_SCRATCH_MIB MiB that the library holds
 * on each GPU it runs on until the process ends; it calls no hipMalloc or
 * hipFree.  Limit: ncols <= CHFSI_NOALLOC_MAX_COLS (CHFSI_ERR_ARG above it);
 * any n_dof (the rotation streams row panels through the array; the overlap
 * uses fewer row splits than chfsi_orthonormalize when its partial tiles
 * would not fit, so results can differ from it in the last bits).  Every call
 * on one GPU uses that GPU's single array: calls that overlap in time on one
 * GPU (from several threads or on several streams) race and must be
 * serialised by the caller.  CHFSI_ERR_STATE if the array's address could not
 * be set up for the context's device (chfsi_create does that once per
 * device). */
#define CHFSI_NOALLOC_MAX_COLS 256
#define CHFSI_NOALLOC_SCRATCH_MIB 96
int chfsi_orthonormalize_noalloc(chfsi_ctx *ctx, double *X, int64_t ld, int ncols, int mixed);

/* ---- rayleighRitz (Sec. 3.5 steps i-iii) ---------------------------------
 * In place, for orthonormal X: HX = Htilde X, Hhat = X^T HX (lower triangle),
 * Hhat Q = Q D (D ascending, FP64 Jacobi on the device), X <- X Q.
 * evals, resid: host arrays [ncols]; resid[i] = ||Htilde x_i - D_i x_i||_2.
 * HX_out (device [n_dof x ld] or NULL) receives Htilde X after rotation. */
int chfsi_rayleigh_ritz(chfsi_ctx *ctx, double *X, int64_t ld, int ncols,
                        double *evals, double *resid, double *HX_out);

/* ---- rayleighRitz with spectrum splitting (Sec. 3.5, Alg. 4, and the
 * mixed-precision projected Hamiltonian of Sec. 3.5, eq.
 * partialDiagMixedPrec1) ---------------------------------------------------
 * For orthonormal X [n_dof x ld] with ncols = N_oc + N_fr columns:
 * HX = Htilde X; Hhat = X^T HX (lower triangle).  mixed = 1: the fr-fr block
 * (rows and columns >= N_oc, its start rounded down to a multiple of 64) in
 * FP64, every other block with FP32 inputs and products; mixed = 0: all FP64.
 * Hhat Q = Q D (FP64 Jacobi; all pairs are computed, the N_fr largest used);
 * the partial rotation X Q_fr goes to Xfr (device [n_dof x ldfr], ldfr >=
 * n_fr, caller-owned, must not overlap X; X is left unchanged, as Alg. 5
 * needs both) or, with Xfr = NULL, over the trailing N_fr columns of X (the
 * first N_oc columns are left as they are).
 * evals_fr, resid_fr: host [n_fr], ascending Ritz values of the N_fr largest
 * pairs and ||Htilde x_i - d_i x_i||_2 of the rotated columns.  Errors:
 * CHFSI_ERR_ARG for n_fr outside 1..ncols, null host arrays, ldfr < n_fr or
 * an Xfr that overlaps X. */
int chfsi_rayleigh_ritz_split(chfsi_ctx *ctx, double *X, int64_t ld, int ncols, int n_fr, int mixed,
                              double *Xfr, int64_t ldfr, double *evals_fr, double *resid_fr);

/* ---- periodic cell and k-points (Sec. 2.1, eq. ksproblemPer) ------------
 * chfsi_set_mesh_periodic: as chfsi_set_mesh on the periodic cell [0, L)^3:
 * node index I = (ex p + a) mod (n_el p), so n = n_el p unknowns per
 * direction and n_dof = (n_el p)^3, no Dirichlet nodes; n_el must be even
 * (>= 2) so that the 8-colour parity rule separates cells that share a node
 * across the wrap.  The real operations (apply, filter, orthonormalize,
 * rayleighRitz, solve) then act on the k = 0 (Gamma point) operator.
 * Errors: CHFSI_ERR_ARG for odd n_el or the set_mesh conditions. */
int chfsi_set_mesh_periodic(chfsi_ctx *ctx, double L, int n_el, int p);

/* chfsi_set_kpoint: the Bloch wave vector k (1/bohr) of the complex operator
 * Htilde_k = M^-1/2 (K - i k.G) M^-1/2 + diag(V + |k|^2/2), G_d the GLL
 * first-derivative matrices int N_j d_d N_l (exactly antisymmetric after the
 * periodic assembly, so Htilde_k is Hermitian).  k = 0 after set_mesh_periodic.
 * Errors: CHFSI_ERR_STATE without a periodic mesh, CHFSI_ERR_ARG for
 * non-finite k. */
int chfsi_set_kpoint(chfsi_ctx *ctx, double kx, double ky, double kz);

/* chfsi_apply_complex: Y = Htilde_k X for complex blocks (interleaved re, im
 * FP64 pairs, i.e. complex128), DoF-major: element (dof i, column j) at
 * X[i*ld + j], ld and ncols in complex elements (ld >= ncols).  X and Y are
 * caller-owned device arrays that must not overlap.  The cell products run on
 * FP64 MFMA as one real contraction of length 2 n_loc per output (A on the
 * columns, B on the swapped (re, im) pairs).  Errors: CHFSI_ERR_STATE without
 * a periodic mesh and potential, CHFSI_ERR_ARG for bad block arguments. */
int chfsi_apply_complex(chfsi_ctx *ctx, const void *X, void *Y, int64_t ld, int ncols);

/* ---- ChFSI at a k-point (Sec. 2.1 eq. ksproblemPer; Sec. 3.3 - 3.5 in their
 * Hermitian form) -------------------------------------------------------------
 * The eigenpairs of the complex Hermitian Htilde_k of chfsi_set_kpoint, on
 * complex128 blocks laid out as for chfsi_apply_complex (ld, ncols in complex
 * elements; caller-owned device arrays).  FP64 throughout.  Every call needs
 * a periodic mesh and a potential (CHFSI_ERR_STATE otherwise) and at most
 * 2048 columns (CHFSI_ERR_ARG).
 * chfsi_get_upper_bound_k: b = sum_d lambda_max(A_{k_d}) + max V, the Weyl
 *   bound of the Kronecker sum of the three 1D Bloch operators plus the
 *   potential (host eigensolve of each 1D operator; above 200 nodes per
 *   direction a Gershgorin bound).
 * chfsi_chebyshev_filter_complex: in place, X <- T_m(Hbar_k) X / T_m(xi0) with
 *   Hbar_k = (Htilde_k - c)/e as for chfsi_chebyshev_filter (real coefficients,
 *   the complex cell kernel); CHFSI_ERR_NONFINITE on NaN/Inf.
 * chfsi_orthonormalize_complex: CholGS in complex arithmetic, S = X^H X =
 *   L L^H, X <- X L^-H (X^H X = I); CHFSI_ERR_NOT_SPD as the real call.
 * chfsi_rayleigh_ritz_complex: for orthonormal X, Hhat = X^H Htilde_k X
 *   (Hermitian), Hhat Q = Q D (D ascending), X <- X Q; evals and resid host
 *   [ncols], resid[i] = ||Htilde_k x_i - D_i x_i||_2; HX_out (device complex
 *   [n_dof x ld] or NULL) receives Htilde_k X.  The projected eigensolve runs
 *   as the real symmetric 2 ncols x 2 ncols form [[Re, Im], [-Im, Re]] (FP64
 *   Jacobi; every eigenvalue appears twice and one complex eigenvector is
 *   taken per pair): CHFSI_ERR_NONFINITE if the pairs cannot be resolved,
 *   CHFSI_WARN_NOT_CONVERGED if the Jacobi sweep cap ended it.
 * chfsi_solve_complex: the loop of chfsi_solve on these steps; opts as there
 *   with no precision ladder beyond FP64 and mixed_cholgs = 0 (CHFSI_ERR_ARG
 *   otherwise); b from chfsi_get_upper_bound_k.  Errors and report as
 *   chfsi_solve. */
int chfsi_get_upper_bound_k(const chfsi_ctx *ctx, double *b);
int chfsi_chebyshev_filter_complex(chfsi_ctx *ctx, void *X, int64_t ld, int ncols, int degree, double a, double b,
                                   double a0, int block_width);
int chfsi_orthonormalize_complex(chfsi_ctx *ctx, void *X, int64_t ld, int ncols);
int chfsi_rayleigh_ritz_complex(chfsi_ctx *ctx, void *X, int64_t ld, int ncols, double *evals, double *resid,
                                void *HX_out);
/* A group of k-points on one periodic mesh (the paper's k-point
 * parallelisation, Sec. 3.7, as one launch per colour): chfsi_set_kpoints
 * takes nk wave vectors (host, 3 nk values, k-point g at k[3g .. 3g+2]) and
 * uploads one cell operator each; chfsi_apply_complex_kpoints computes
 * Y_g = Htilde_{k_g} X_g for all g, block g at X + g*stride (and Y + g*stride),
 * stride in complex elements (>= n_dof * ld), layout as chfsi_apply_complex.
 * Work items (k-point, cell, column tile) share the mesh tables.  A new mesh
 * clears the group.  Errors: CHFSI_ERR_STATE without a periodic mesh (or
 * without a group for the apply), CHFSI_ERR_ARG for nk < 1, non-finite k,
 * stride < n_dof * ld or overlapping X and Y. */
int chfsi_set_kpoints(chfsi_ctx *ctx, int nk, const double *k);
int chfsi_apply_complex_kpoints(chfsi_ctx *ctx, const void *X, void *Y, int64_t ld, int ncols, int64_t stride);

/* ---- electrostatics: the discrete Poisson problem (Sec. 2.4 eq.
 * phiTotDiscreteSolve), homogeneous Dirichlet conditions ------------------
 * A phi = f with A = 1/(4 pi) int grad N_i . grad N_j on the mesh's GLL
 * elements and f = M rho + q (the GLL rule makes int rho N_i = M_ii rho_i; a
 * point charge q_I on node d_I adds q_I to f_{d_I}: the paper's nuclear
 * charges b_I = -Z_I delta sit on nodes).  On the uniform mesh A is applied
 * matrix-free as the Kronecker sum of the banded 1D stiffness and the 1D
 * masses (the assembled form of the paper's matrix-free operator).
 * chfsi_poisson_apply: y = A x (device [n_dof] each, not overlapping).
 * chfsi_poisson_solve: Jacobi-preconditioned conjugate gradients (the paper's
 * solver, Sec. 3.2) from the initial guess in phi (device [n_dof], in/out) to
 * ||f - A phi|| <= tol ||f||; rho device [n_dof] (Dirichlet nodes carry no
 * DoF); charge_dofs/charges host [ncharges] (charges on one node add up).
 * iters and rel_resid (the true residual of the returned phi, recomputed at
 * the end) may be NULL.  Returns 0, or CHFSI_WARN_NOT_CONVERGED when max_iter
 * ends the iteration first.  Needs a mesh (no potential); CHFSI_ERR_STATE on
 * a periodic mesh (a periodic cell needs a neutral charge); CHFSI_ERR_ARG for
 * bad pointers, tol <= 0 or a charge dof outside 0..n_dof-1. */
int chfsi_poisson_apply(chfsi_ctx *ctx, const double *x, double *y);
int chfsi_poisson_solve(chfsi_ctx *ctx, const double *rho, int ncharges, const int64_t *charge_dofs,
                        const double *charges, double *phi, double tol, int max_iter, int *iters, double *rel_resid);

/* ---- Fermi energy (Alg. 5 step 1) ------------------------------------------
 * The mu at which 2 (n_oc + sum_k f(evals_fr[k], mu)) = n_electrons, with the
 * Fermi-Dirac occupancy f(e, mu) = 1 / (1 + exp((e - mu) / sigma)) of Sec. 2.1
 * (sigma = k_B T in Hartree).  Pure host function (no context, no device):
 * bisection on the monotone count to the last representable midpoint.
 * Errors: CHFSI_ERR_ARG for null pointers, n_fr < 1, n_oc < 0, sigma <= 0,
 * non-finite values, or n_electrons outside (2 n_oc, 2 (n_oc + n_fr)). */
int chfsi_fermi_level(const double *evals_fr, int n_fr, int n_oc, double n_electrons, double sigma, double *mu);

/* ---- electron density (Alg. 5 steps 2-3, eq. elecDensSP) -----------------
 * With the collocated GLL quadrature the basis functions are the nodes'
 * Lagrange polynomials, so the density at interior node j is
 *   rho[j] = 2 M_jj^-1 ( sum_{i<ncols} X[j,i]^2
 *                        + sum_{k<n_fr} (f(evals_fr[k], mu) - 1) Xfr[j,k]^2 ),
 * X the orthonormal basis (Psi^o, all N = N_oc + N_fr columns, unrotated),
 * Xfr = X Q_fr from chfsi_rayleigh_ritz_split (out of place), evals_fr its
 * host Ritz values.  n_fr = 0 gives the fully occupied density (Xfr and
 * evals_fr unused).  rho: device [n_dof], caller-owned; Dirichlet nodes carry
 * no DoF and have zero density.  One wave per DoF row, HBM-bound.  Errors:
 * CHFSI_ERR_ARG for bad block arguments, n_fr > 0 without Xfr/evals_fr or
 * with ldfr < n_fr, sigma <= 0 when n_fr > 0, or a null rho. */
int chfsi_density(chfsi_ctx *ctx, const double *X, int64_t ld, int ncols, const double *Xfr, int64_t ldfr,
                  int n_fr, const double *evals_fr, double mu, double sigma, double *rho);

/* ---- solve (Alg. 2 step 7 with the adaptive repeat of Sec. 3.3) ----------
 * X: device [n_dof x ld], ld >= nblock, holds the start (or warm-start) block
 * on entry and the Ritz vectors (tilde space, orthonormal) on exit.
 * Loop: CholGS + RR on X; then repeat {filter (a = largest Ritz value, b from
 * set_potential, a0 = smallest), CholGS, RR} until
 * max_{i < nstates} resid_i <= tol or max_iter filter passes.
 * evals, resid: host [nblock].  rep (may be NULL) receives counters/timings.
 * The filter precision follows the ladder: rung k (ladder[k]) is left for
 * rung k+1 when the largest wanted residual drops below ladder_tol[k], or
 * stagnates (a pass reduces it by less than 2 %).  ladder_tol[k] <= 0 selects
 * 4 u_k b, with u_k the unit roundoff of the rung's products (BF16 2^-8,
 * BF16X3 2^-16, FP32 2^-24) and b the spectral upper bound: a reduced-
 * precision filter leaves residuals of about u ||Htilde||.  n_ladder = 0 means
 * FP64 throughout.  mixed_cholgs selects the paper's mixed CholGS
 * (eq. overlapmixedprec) on every rung but the last one of a ladder of two or
 * more rungs (with n_ladder <= 1: throughout). */
typedef struct {
    int nstates;          /* wanted states N                                  */
    int nblock;           /* block size N_b >= nstates (guard states)         */
    int degree;           /* Chebyshev degree m                               */
    int max_iter;         /* cap on filter passes                             */
    int block_width;      /* filter block width (0 = default)                 */
    double tol;           /* residual tolerance on the wanted states          */
    chfsi_prec ladder[4]; /* filter precision ladder                          */
    int n_ladder;
    double ladder_tol[4]; /* residual that ends rung k (<= 0: 4 u_k b)         */
    int mixed_cholgs;     /* 1: paper's mixed CholGS                          */
} chfsi_opts;

typedef struct {
    int iters;            /* filter passes done                               */
    int status;           /* same as the return value                         */
    int rung;             /* ladder rung in use at exit                       */
    double t_filter, t_cholgs, t_rr;   /* seconds (device events)              */
    double max_resid;     /* largest wanted residual at exit                  */
    int64_t dofvecs;      /* Htilde applications x n_dof                      */
} chfsi_report;

int chfsi_solve(chfsi_ctx *ctx, const chfsi_opts *o, double *X, int64_t ld,
                double *evals, double *resid, chfsi_report *rep);
/* The solve on the complex Bloch operator at the context's k-point (see
 * chfsi_solve_complex above). */
int chfsi_solve_complex(chfsi_ctx *ctx, const chfsi_opts *o, void *X, int64_t ld,
                        double *evals, double *resid, chfsi_report *rep);

/* ---- solveBatch (many independent problems; the paper's k-point groups,
 * Sec. 3.7, placed on one device) ---------------------------------------------
 * ctxs[i] holds problem i's mesh and potential (one context per problem, all
 * on the same device; distinct streams let the per-problem CholGS/RR overlap).
 * Every problem uses the same Chebyshev degree; each follows its own ladder
 * of BF16, BF16X3, FP32 and FP64 filter rungs (CholGS/RR are FP64; BF16 rungs
 * need p <= 7, else CHFSI_ERR_ARG).  Each pass runs one
 * Chebyshev step of all active problems in shared launches (one per padded
 * cell size and colour) captured once per active set in a HIP graph, then
 * CholGS + RR per problem on host threads; a problem leaves the batch when its
 * wanted residuals are <= opts[i].tol or after opts[i].max_iter passes.
 * X[i]: device [n_dof_i x ld[i]] start block in, Ritz vectors out;
 * evals[i], resid[i]: host [nblock_i]; reps (may be NULL) [n].
 * Returns CHFSI_WARN_NOT_CONVERGED if any problem did not converge or failed;
 * reps[i].status then tells which (< 0: that problem's own error, see
 * chfsi_batch_pass). */
int chfsi_solve_batch(chfsi_ctx *const *ctxs, int n, const chfsi_opts *opts, double *const *X,
                      const int64_t *ld, double *const *evals, double *const *resid, chfsi_report *reps);

/* ---- batch session (continuous batching) ----------------------------------
 * A session holds a changing set of problems that share the batched sweeps of
 * chfsi_solve_batch.  chfsi_batch_add puts a problem in (its context, options,
 * block and host result arrays must stay valid until it leaves); it starts at
 * the next pass with CholGS + RR of its block (a warm start needs nothing
 * else).  chfsi_batch_pass runs one pass for every problem in the session:
 * a degree-m filter (problems on a BF16 or BF16X3 rung share one
 * graph-captured sweep, problems on their FP32 rung another, problems on the
 * FP64 rung a third), then CholGS + RR per problem;
 * problems whose wanted residuals are <= tol, or that reached max_iter, leave
 * and their ids are written to done_ids (at most max_done; the rest are
 * reported by later calls).  Each problem follows its own precision ladder
 * (rung thresholds as in chfsi_solve).
 * A problem's results do not depend on which other problems share its passes.
 * A problem whose own step fails leaves the session with that status in its
 * report (rep.status < 0) and its id in done_ids, while the others go on:
 * CHFSI_ERR_NONFINITE when its Ritz values give no valid filter bounds
 * (a0 < a < b), CHFSI_ERR_NOT_SPD from its CholGS, CHFSI_ERR_HIP from a call on
 * its stream.  chfsi_batch_pass itself returns an error only for a failure of
 * the shared work (the graph-captured sweep, the batched eigensolve). */
typedef struct chfsi_batch chfsi_batch;
int chfsi_batch_create(chfsi_batch **out, int device);
int chfsi_batch_destroy(chfsi_batch *b);
/* returns the problem id (>= 0) or an error status (< 0) */
int chfsi_batch_add(chfsi_batch *b, chfsi_ctx *ctx, const chfsi_opts *o, double *X, int64_t ld,
                    double *evals, double *resid);
/* returns the number of problems still in the session (>= 0) or an error */
int chfsi_batch_pass(chfsi_batch *b, int *done_ids, int *n_done, int max_done);
int chfsi_batch_report(const chfsi_batch *b, int id, chfsi_report *rep);
const char *chfsi_batch_last_error(const chfsi_batch *b);
/* Host threads that run the per-problem CholGS / Rayleigh-Ritz steps of a
 * pass (default 8).  Problems whose contexts share a HIP stream are always
 * handled by one thread in turn, so no stream is driven by two threads at
 * once; threads = 1 runs every problem from the calling thread (for tracers
 * and debuggers).  A new session (also the one chfsi_solve_batch makes) takes
 * its default from the environment variable CHFSI_BATCH_THREADS when set to
 * 1..256.  Errors: CHFSI_ERR_ARG outside 1..256. */
int chfsi_batch_set_threads(chfsi_batch *b, int threads);
/* Device bytes a context holds once it is in a batch session with nblock
 * vectors (mesh and potential tables, the CholGS / Rayleigh-Ritz workspaces,
 * three FP64-sized recursion buffers and HX), not counting the caller's block
 * (pure; no device access; 0 for arguments outside the supported range). */
size_t chfsi_batch_footprint_bytes(int n_el, int p, int nblock);

/* ---- admission / diagnostics ---------------------------------------------
 * Device bytes a context needs for (n_el, p) and a solve of nblock vectors with
 * the given filter block width and precision (pure; no device access). */
size_t chfsi_footprint_bytes(int n_el, int p, int nblock, int block_width, chfsi_prec prec);
/* Device bytes the context holds right now (its buffers only grow until
 * destroy, so a reused context may hold more than a new problem needs). */
int chfsi_device_bytes(const chfsi_ctx *ctx, size_t *bytes);
const char *chfsi_status_string(int status);
const char *chfsi_last_error(const chfsi_ctx *ctx);
/* Timing of the cell-product kernel (the filter's dominant kernel): when
 * enabled, every launch of it is bracketed by HIP events on the context
 * stream.  chfsi_last_filter_timing synchronises the stream and returns the
 * summed device time (ms) and the launch count since the last reset, plus
 * the cell-product work in those launches as cell-vector products
 * (cells x columns, so flops = 2 n_loc^2 x that count). */
int chfsi_set_timing(chfsi_ctx *ctx, int enable);
int chfsi_reset_timing(chfsi_ctx *ctx);
int chfsi_last_filter_timing(chfsi_ctx *ctx, double *ms_cells, int *n_launches, int64_t *cell_vecs);
/* Tile configuration of the cell-product kernel (the filter's work-group
 * shape; Sec. 3.3 leaves the blocking of the cell-level products to the
 * implementation): -1 = built-in choice (default), 0 = four waves with two
 * 16-column blocks each, 1 = eight waves with one block each (more resident
 * waves, fewer accumulators).  Every variant computes the same products; an
 * autotuner times them per degree and precision and sets the faster.
 * Applies to later filter/apply calls and to batch sweeps built after it
 * (set it before adding the context to a batch session).  Errors:
 * CHFSI_ERR_ARG for a null ctx or a variant outside -1..1. */
int chfsi_set_tile_variant(chfsi_ctx *ctx, int variant);
/* Cells per work-group of the FP64/FP32 cell-product kernel (p <= 6; one
 * cell above): the tile's 64 columns are split over 1, 2 or 4 cells of one
 * colour, so a block of few columns pads fewer of them (24 columns fill a
 * 64-column tile to 37 %, and two 16-column groups of four cells to 75 %);
 * 0 (default) picks the count that pads the fewest columns, ties to fewer
 * cells.  Every setting computes the same products.  Applies to later
 * filter/apply calls and to batch sweeps built after it.  Errors:
 * CHFSI_ERR_ARG for a value other than 0, 1, 2, 4. */
int chfsi_set_cells_per_tile(chfsi_ctx *ctx, int cpt);
/* How rayleighRitz (both forms) obtains Htilde times the rotated columns for
 * the residuals (Sec. 3.5 step iii leaves this open): 0 = cost model
 * (default): rotate HX with X when that GEMM is cheaper than the cell
 * products, else apply Htilde again; 1 = always rotate HX; 2 = always apply
 * Htilde again.  Both give the same vectors up to rounding; HX_out receives
 * whichever.  Errors: CHFSI_ERR_ARG for a null ctx or a mode outside 0..2. */
int chfsi_set_rr_residual(chfsi_ctx *ctx, int mode);
/* Cap on the Jacobi sweeps of the projected eigensolve (Sec. 3.5 step ii;
 * default 40; a filtered block needs about 10).  When the cap ends the
 * eigensolve before its off-diagonal norm meets the tolerance, rayleighRitz
 * (both forms) returns CHFSI_WARN_NOT_CONVERGED with the last iterate's pairs,
 * and a solve or batch problem whose last Rayleigh-Ritz did so reports
 * CHFSI_WARN_NOT_CONVERGED.  Errors: CHFSI_ERR_ARG outside 1..1000. */
int chfsi_set_jacobi_sweeps(chfsi_ctx *ctx, int max_sweeps);

#ifdef __cplusplus
}
#endif
#endif /* CHFSI_H */
