// ChFSI on the complex Hermitian Bloch operator at a k-point (Sec. 2.1 eq.
// ksproblemPer; the steps of Sec. 3.3 - 3.5 in their Hermitian form).
//
// A complex block X (n_dof x N, interleaved re/im) is handled as the real
// block R (n_dof x 2N) of its interleaved columns, so the dense subspace
// products reuse the real MFMA kernels with no extra arithmetic:
//  * the overlap X^H X and the projection X^H (H X) come from the real Gram
//    R^T B of 2N columns (the same flop count as the complex products) and
//    are folded into the real 2N x 2N embedding emb(M) (2 x 2 blocks
//    [[Re, Im], [-Im, Re]]);
//  * the Cholesky factor of emb(S) is emb(L) (S = L L^H, L with a real
//    positive diagonal: real Cholesky is unique), and its inverse transpose
//    is emb(L^-H), so R emb(L^-H) is X L^-H -- the complex CholGS;
//  * the projected eigenproblem is solved as the real symmetric emb(Hhat),
//    whose eigenvalues are those of Hhat, each twice; a selection kernel
//    picks one complex eigenvector per pair (herm_select_launch) and builds
//    emb(Q), so the rotation R emb(Q) is X Q.
// The Chebyshev filter is the real recursion with the complex cell kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/chfsi.h"
#include "ctx.hpp"
#include "kernels.hpp"

namespace chfsi {

// E = emb(M), M Hermitian from the lower triangle of G (see kernels.hpp).
__global__ __launch_bounds__(256) void herm_embed_kernel(const double *__restrict__ G, int n2,
                                                         double *__restrict__ E) {
  const int64_t total = (int64_t)n2 * n2;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / n2), col = (int)(t - (int64_t)r * n2);
    const int j = r >> 1, a = r & 1, k = col >> 1, b = col & 1;
    const int hi = j > k ? j : k, lo = j > k ? k : j;     // entry (hi, lo) of the lower triangle
    const double re = G[(int64_t)(2 * hi) * n2 + 2 * lo] + G[(int64_t)(2 * hi + 1) * n2 + 2 * lo + 1];
    double im = 0.0;
    if (hi != lo) {
      im = G[(int64_t)(2 * hi) * n2 + 2 * lo + 1] - G[(int64_t)(2 * hi + 1) * n2 + 2 * lo];
      if (j < k) im = -im;                                 // M_jk = conj(M_kj)
    }
    // emb(re + i im) = [[re, im], [-im, re]]
    E[t] = (a == b) ? re : (a == 0 ? im : -im);
  }
}

void herm_embed_launch(const double *G, int n2, double *E, hipStream_t s) {
  int64_t blocks = ((int64_t)n2 * n2 + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) return;
  hipLaunchKernelGGL(herm_embed_kernel, dim3((unsigned)blocks), dim3(256), 0, s, G, n2, E);
}

static constexpr int SEL_MAX = 4096;
static constexpr int SEL_T = 1024;

__global__ __launch_bounds__(SEL_T) void herm_select_kernel(const double *__restrict__ V,
                                                            const double *__restrict__ ev, int n2,
                                                            double *__restrict__ Q, double *__restrict__ evals,
                                                            double *__restrict__ lam2, int *__restrict__ status) {
  __shared__ double v[SEL_MAX];
  __shared__ double cf[SEL_MAX];
  __shared__ double red[SEL_T / 64];
  __shared__ double nrm_s;
  const int t = threadIdx.x;
  const int N = n2 / 2;
  int kept = 0;
  for (int i = 0; i < n2 && kept < N; ++i) {
    for (int r = t; r < n2; r += SEL_T) v[r] = V[(int64_t)r * n2 + i];
    __syncthreads();
    const int m2 = 2 * kept;
    for (int pass = 0; pass < 2 && m2 > 0; ++pass) {
      // coefficients against the kept columns, then their removal
      for (int m = t; m < m2; m += SEL_T) {
        double acc = 0.0;
        for (int r = 0; r < n2; ++r) acc += Q[(int64_t)r * n2 + m] * v[r];
        cf[m] = acc;
      }
      __syncthreads();
      for (int r = t; r < n2; r += SEL_T) {
        double acc = 0.0;
        for (int m = 0; m < m2; ++m) acc += Q[(int64_t)r * n2 + m] * cf[m];
        v[r] -= acc;
      }
      __syncthreads();
    }
    double part = 0.0;
    for (int r = t; r < n2; r += SEL_T) part += v[r] * v[r];
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
    if ((t & 63) == 0) red[t >> 6] = part;
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int w = 0; w < SEL_T / 64; ++w) s += red[w];
      nrm_s = sqrt(s);
    }
    __syncthreads();
    const double nrm = nrm_s;
    if (nrm > 0.1) {
      const double inv = 1.0 / nrm;
      for (int r = t; r < n2; r += SEL_T) {
        const double jv = (r & 1) ? v[r - 1] : -v[r + 1];   // (Jv)_2j = -v_2j+1, (Jv)_2j+1 = v_2j
        Q[(int64_t)r * n2 + m2] = v[r] * inv;
        Q[(int64_t)r * n2 + m2 + 1] = jv * inv;
      }
      if (t == 0) {
        evals[kept] = ev[i];
        lam2[m2] = ev[i];
        lam2[m2 + 1] = ev[i];
      }
      ++kept;
    }
    __syncthreads();
  }
  if (t == 0) *status = kept;
}

void herm_select_launch(const double *V, const double *ev, int n2, double *Q, double *evals, double *lam2,
                        int *status, hipStream_t s) {
  hipLaunchKernelGGL(herm_select_kernel, dim3(1), dim3(SEL_T), 0, s, V, ev, n2, Q, evals, lam2, status);
}

}  // namespace chfsi

using namespace chfsi;

namespace {

int check_complex(chfsi_ctx *c, const void *X, int64_t ld, int ncols) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (!c->mesh.periodic) return fail(c, CHFSI_ERR_STATE, "complex ChFSI: needs a periodic mesh (set_mesh_periodic)");
  if (2 * ncols > SEL_MAX) return fail(c, CHFSI_ERR_ARG, "complex ChFSI: at most 2048 columns");
  return 0;
}

// Y = s1 (Htilde_k - shift) X + s2 Xp on complex blocks (ld, ncols in complex elements).
int cheb_step_c(chfsi_ctx *c, const double *X, int64_t ldx, const double *Xp, int64_t ldp, double *Y, int64_t ldy,
                int ncols, double s1, double s2, double shift) {
  const MeshTables &M = c->mesh;
  HxArgs<double> a;
  a.X = X;
  a.ldx = 2 * ldx;
  a.Xp = Xp;
  a.ldp = 2 * ldp;
  a.Y = Y;
  a.ldy = 2 * ldy;
  a.K = c->Kc64.as<double>();
  a.cmap = c->cmap.as<int32_t>();
  a.n_loc = M.n_loc;
  a.np = M.np;
  a.q = M.q;
  a.n_el = M.n_el;
  a.cells = c->cells.as<int32_t>();
  a.minv = c->minv64.as<double>();
  a.V = c->V64.as<double>();
  a.ncols = 2 * ncols;
  a.s1 = s1;
  a.s2 = s2;
  // the diagonal of Htilde_k is V + |k|^2 / 2; the epilogue adds s1 (V - shift) X
  a.shift = shift - 0.5 * (c->kvec[0] * c->kvec[0] + c->kvec[1] * c->kvec[1] + c->kvec[2] * c->kvec[2]);
  a.variant = c->tile_variant;
  for (int col = 0; col < 8; ++col)
    if (hx_cells_cplx_launch(a, M.color_offset[col], M.color_offset[col + 1], c->stream) != 0)
      return fail(c, CHFSI_ERR_ARG, "complex step: unsupported cell size");
  if (c->timing) c->cell_vecs += (int64_t)M.n_cells * 2 * ncols;
  HIPCHK(c, hipGetLastError());
  return 0;
}

int filter_c(chfsi_ctx *c, double *X, int64_t ld, int ncols, int degree, double a, double b, double a0, int bw) {
  const double cc = 0.5 * (a + b), e = 0.5 * (b - a), xi0 = (a0 - cc) / e;
  const int64_t nd = c->mesh.n_dof;
  bw = std::min(bw > 0 ? bw : 64, ncols);
  for (int i = 0; i < 3; ++i) HIPCHK(c, c->fbuf[i].ensure((size_t)nd * bw * 16));
  for (int j0 = 0; j0 < ncols; j0 += bw) {
    const int w = std::min(bw, ncols - j0);
    double *buf[3] = {X + 2 * j0, c->fbuf[1].as<double>(), c->fbuf[2].as<double>()};
    const int64_t lds[3] = {ld, w, w};
    int cur = 0, prev = -1;
    double rho = 1.0 / xi0;
    for (int k = 0; k < degree; ++k) {
      double s1, s2;
      if (k == 0) {
        s1 = rho / e;
        s2 = 0.0;
      } else {
        const double rn = 1.0 / (2.0 * xi0 - rho);
        s1 = 2.0 * rn / e;
        s2 = -rn * rho;
        rho = rn;
      }
      int out = 0;
      while (out == cur || out == prev) ++out;
      if (int r = cheb_step_c(c, buf[cur], lds[cur], prev >= 0 ? buf[prev] : nullptr, prev >= 0 ? lds[prev] : 0,
                              buf[out], lds[out], w, s1, s2, cc))
        return r;
      prev = cur;
      cur = out;
    }
    // complex w columns are 2 w doubles
    if (cur != 0) copy_cols_launch<double, double>(buf[cur], 2 * lds[cur], X + 2 * j0, 2 * ld, nd, 2 * w, c->stream);
  }
  HIPCHK(c, c->flag.ensure(4 * sizeof(int)));
  zero_int_launch(c->flag.as<int>(), 1, c->stream);
  nonfinite_launch<double>(X, 2 * ld, nd, 2 * ncols, c->flag.as<int>(), c->stream);
  int hflag = 0;
  HIPCHK(c, hipMemcpyAsync(&hflag, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (hflag) return fail(c, CHFSI_ERR_NONFINITE, "complex filter produced NaN/Inf (upper bound below lambda_max?)");
  return 0;
}

// Rayleigh-Ritz on the complex block X (N columns), HX a complex buffer.
int rr_c(chfsi_ctx *c, double *X, int64_t ld, int N, double *HX, int64_t ldh, double *evals, double *resid) {
  const int64_t nd = c->mesh.n_dof;
  const int n2 = 2 * N;
  if (int r = ensure_small(c, n2)) return r;
  HIPCHK(c, c->csel.ensure((size_t)N * sizeof(double) + 16));
  // step i: HX = Htilde_k X, Hhat = X^H HX (as the embedding of the real Gram)
  if (int r = cheb_step_c(c, X, ld, nullptr, 0, HX, ldh, N, 1.0, 0.0, 0.0)) return r;
  gram_launch(X, 2 * ld, HX, 2 * ldh, nd, n2, c->gram_part.as<double>(), c->Zmat.as<double>(), 0, c->stream);
  herm_embed_launch(c->Zmat.as<double>(), n2, c->Smat.as<double>(), c->stream);
  // step ii: eigenpairs of emb(Hhat), one complex eigenvector per pair
  const JacobiJob job = rr_eigen_job(c, n2);
  const int jr = jacobi_eigh(job.A, n2, job.work, job.evals, job.Q, 1e-14, c->jac_sweeps, c->host_scratch.data(),
                             c->stream, nullptr);
  if (jr < 0) return fail(c, CHFSI_ERR_HIP, "Jacobi eigensolver: HIP error");
  double *ev_c = c->csel.as<double>();
  int *kept_d = reinterpret_cast<int *>(ev_c + N);
  double *lam2 = c->diag0.as<double>();
  double *Qe = c->Zmat.as<double>();
  herm_select_launch(job.Q, job.evals, n2, Qe, ev_c, lam2, kept_d, c->stream);
  int kept = 0;
  HIPCHK(c, hipMemcpyAsync(&kept, kept_d, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (kept != N) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "complex Rayleigh-Ritz: %d of %d eigenvector pairs resolved", kept, N);
    return fail(c, CHFSI_ERR_NONFINITE, msg);
  }
  // step iii: X <- X Q; Htilde_k on the rotated columns by rotating HX or a fresh application
  double *scr = c->rscratch.as<double>();
  const size_t se = c->rscratch.bytes / sizeof(double);
  if (rmul_cols_launch(X, 2 * ld, nd, n2, Qe, n2, n2, 0, 0, 0, scr, se, c->stream) != 0)
    return fail(c, CHFSI_ERR_ARG, "complex Rayleigh-Ritz: block too wide for the row-panel kernel");
  if (rr_reapply(c, N)) {
    if (int r = cheb_step_c(c, X, ld, nullptr, 0, HX, ldh, N, 1.0, 0.0, 0.0)) return r;
  } else if (rmul_cols_launch(HX, 2 * ldh, nd, n2, Qe, n2, n2, 0, 0, 0, scr, se, c->stream) != 0) {
    return fail(c, CHFSI_ERR_ARG, "complex Rayleigh-Ritz: block too wide for the row-panel kernel");
  }
  // residuals of the real and imaginary columns, combined per complex column
  resid_launch(X, 2 * ld, HX, 2 * ldh, lam2, nd, n2, c->resid_part.as<double>(), c->resid_d.as<double>(), c->stream);
  std::vector<double> r2(n2);
  HIPCHK(c, hipMemcpyAsync(evals, ev_c, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(r2.data(), c->resid_d.p, n2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < N; ++k) resid[k] = std::hypot(r2[2 * k], r2[2 * k + 1]);
  HIPCHK(c, hipGetLastError());
  return jr > 0 ? jacobi_warning(c) : 0;
}

}  // namespace

extern "C" int chfsi_chebyshev_filter_complex(chfsi_ctx *c, void *X, int64_t ld, int ncols, int degree, double a,
                                              double b, double a0, int block_width) {
  if (int r = check_complex(c, X, ld, ncols)) return r;
  if (degree < 0 || !(a0 < a) || !(a < b)) return fail(c, CHFSI_ERR_ARG, "filter: need a0 < a < b, degree >= 0");
  if (degree == 0) return 0;
  return filter_c(c, static_cast<double *>(X), ld, ncols, degree, a, b, a0, block_width);
}

extern "C" int chfsi_orthonormalize_complex(chfsi_ctx *c, void *X, int64_t ld, int ncols) {
  if (int r = check_complex(c, X, ld, ncols)) return r;
  int passes = 0;
  return orth_robust(c, static_cast<double *>(X), 2 * ld, 2 * ncols, 0, &passes, true);
}

extern "C" int chfsi_rayleigh_ritz_complex(chfsi_ctx *c, void *X, int64_t ld, int ncols, double *evals,
                                           double *resid, void *HX_out) {
  if (int r = check_complex(c, X, ld, ncols)) return r;
  if (!evals || !resid) return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz_complex: evals/resid must be host arrays");
  double *HX = static_cast<double *>(HX_out);
  int64_t ldh = ld;
  if (!HX) {
    HIPCHK(c, c->HX.ensure((size_t)c->mesh.n_dof * ncols * 16));
    HX = c->HX.as<double>();
    ldh = ncols;
  }
  if (HX == X) return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz_complex: HX_out must not alias X");
  return rr_c(c, static_cast<double *>(X), ld, ncols, HX, ldh, evals, resid);
}

extern "C" int chfsi_solve_complex(chfsi_ctx *c, const chfsi_opts *o, void *Xv, int64_t ld, double *evals,
                                   double *resid, chfsi_report *rep) {
  if (!o) return fail(c, CHFSI_ERR_ARG, "solve_complex: null options");
  const int nb = o->nblock;
  if (int r = check_complex(c, Xv, ld, nb)) return r;
  if (o->nstates < 1 || o->nstates > nb || o->degree < 1 || o->max_iter < 0 || !(o->tol > 0) || !evals || !resid)
    return fail(c, CHFSI_ERR_ARG, "solve_complex: invalid options");
  if (o->mixed_cholgs || (o->n_ladder > 0 && (o->n_ladder > 1 || o->ladder[0] != CHFSI_FP64)))
    return fail(c, CHFSI_ERR_ARG, "solve_complex: FP64 only (no precision ladder, no mixed CholGS)");
  if (nb > c->mesh.n_dof) return fail(c, CHFSI_ERR_ARG, "solve_complex: more vectors than degrees of freedom");
  double *X = static_cast<double *>(Xv);
  HIPCHK(c, c->HX.ensure((size_t)c->mesh.n_dof * nb * 16));
  double *HX = c->HX.as<double>();
  const double b = c->kin_k + c->vmax;
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i) HIPCHK(c, hipEventCreate(&ev[i]));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int i = 0; i < 6; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  auto secs = [](hipEvent_t x, hipEvent_t y) {
    float ms = 0;
    return hipEventElapsedTime(&ms, x, y) == hipSuccess ? ms * 1e-3 : 0.0;
  };
  chfsi_report R;
  std::memset(&R, 0, sizeof R);
  int passes = 0;
  HIPCHK(c, hipEventRecord(ev[0], c->stream));
  if (int st = orth_robust(c, X, 2 * ld, 2 * nb, 0, &passes, true)) return st;
  HIPCHK(c, hipEventRecord(ev[1], c->stream));
  int rr_st = rr_c(c, X, ld, nb, HX, nb, evals, resid);
  if (rr_st < 0) return rr_st;
  HIPCHK(c, hipEventRecord(ev[2], c->stream));
  HIPCHK(c, hipEventSynchronize(ev[2]));
  R.t_cholgs += secs(ev[0], ev[1]);
  R.t_rr += secs(ev[1], ev[2]);
  R.dofvecs += c->mesh.n_dof * (int64_t)nb;
  auto maxres = [&]() {
    double m = 0;
    for (int i = 0; i < o->nstates; ++i) m = std::max(m, resid[i]);
    return m;
  };
  double res = maxres();
  int it = 0;
  while (res > o->tol && it < o->max_iter) {
    const double a = evals[nb - 1], a0 = evals[0];
    if (!(a0 < a && a < b)) return fail(c, CHFSI_ERR_NONFINITE, "solve_complex: Ritz values outside the filter bounds");
    HIPCHK(c, hipEventRecord(ev[3], c->stream));
    if (int st = filter_c(c, X, ld, nb, o->degree, a, b, a0, o->block_width)) return st;
    HIPCHK(c, hipEventRecord(ev[4], c->stream));
    if (int st = orth_robust(c, X, 2 * ld, 2 * nb, 0, &passes, true)) return st;
    HIPCHK(c, hipEventRecord(ev[5], c->stream));
    rr_st = rr_c(c, X, ld, nb, HX, nb, evals, resid);
    if (rr_st < 0) return rr_st;
    HIPCHK(c, hipEventRecord(ev[0], c->stream));
    HIPCHK(c, hipEventSynchronize(ev[0]));
    R.t_filter += secs(ev[3], ev[4]);
    R.t_cholgs += secs(ev[4], ev[5]);
    R.t_rr += secs(ev[5], ev[0]);
    R.dofvecs += c->mesh.n_dof * (int64_t)nb * (o->degree + 1);
    ++it;
    res = maxres();
    if (c->verbose) {
      std::fprintf(stderr, "[chfsi] complex pass %d: max wanted residual %.3e\n", it, res);
      std::fflush(stderr);
    }
  }
  R.iters = it;
  R.max_resid = res;
  R.status = (res <= o->tol && rr_st == 0) ? CHFSI_OK : CHFSI_WARN_NOT_CONVERGED;
  if (rep) *rep = R;
  return R.status;
}
