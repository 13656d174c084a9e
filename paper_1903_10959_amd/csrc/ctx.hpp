// Internal: the context object behind the opaque chfsi_ctx handle and the
// helpers shared by the single-problem (context.hip) and batched (batch.hip)
// drivers.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/chfsi.h"
#include "kernels.hpp"
#include "mesh.hpp"

namespace chfsi {

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t want) {
    if (want <= bytes) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      bytes = 0;
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) bytes = want;
    else p = nullptr;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};


}  // namespace chfsi

struct chfsi_ctx {
  int device = 0;           // -1: host-only context (tables only, no device work)
  hipStream_t stream = nullptr;
  std::string err;
  chfsi::MeshTables mesh;
  bool has_mesh = false, has_pot = false;
  double vmax = 0, ub = 0;
  // device tables
  chfsi::DevBuf cmap, cells, K64, K32, minv64, minv32, V64, V32, Kbh, Kbl;
  int npb = 0;   // n_loc rounded up to 32 (BF16 tiles); 0 above p = 7 (no BF16 kernel)
  int kc_stride = 0;  // row stride of the padded cell matrix K64 / K32
  int tile_variant = -1;  // cell-kernel tile configuration (-1: built-in choice)
  int cpt_setting = 0;    // cells per work-group of the cell kernel (0: chosen from the column count)
  int rr_residual = 0;    // Ritz residuals: 0 cost model, 1 rotate HX, 2 apply Htilde again
  int jac_sweeps = 40;    // cap on Jacobi sweeps of the projected eigensolve
  // workspaces
  chfsi::DevBuf fbuf[3];      // filter recursion buffers
  chfsi::DevBuf occ_d;    // density: fr occupancy weights
  chfsi::DevBuf Kc64;     // periodic mesh: [A ; (k.G)^T] complex cell operator, 2 np x np
  double kvec[3] = {0, 0, 0};
  double kin_k = 0;       // sum over directions of lambda_max of the 1D Bloch operators at kvec
  chfsi::DevBuf csel;     // complex Rayleigh-Ritz: selected Ritz values and the pairing status
  chfsi::DevBuf Kcg, kshift; // k-point group: nk cell operators and |k|^2/2 shifts
  // Poisson: 1D band / mass tables (for the mesh they were built for), CG
  // workspace, point charges
  chfsi::DevBuf pois_kb, pois_m, pois_work, pois_q;
  int pois_n = 0, pois_p = 0;
  double pois_h = 0;
  int nk = 0;
  std::vector<double> kgroup;
  chfsi::DevBuf gram_part, Smat, dinv, Zmat, Wmat, jac_work, evals_d, resid_part, resid_d, flag, HX, diag0, minratio,
      rscratch;
  std::vector<double> host_scratch = std::vector<double>(16);
  // timing of the cell-product launches
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  int64_t cell_vecs = 0;
  bool verbose = false;   // CHFSI_VERBOSE: one progress line per solve pass on stderr
  // every device buffer the context owns
  template <typename F> void each_buf(F f) {
    chfsi::DevBuf *all[] = {&cmap, &cells, &K64, &K32, &minv64, &minv32, &V64, &V32, &Kbh, &Kbl, &fbuf[0],
                            &fbuf[1], &fbuf[2], &gram_part, &Smat, &dinv, &Zmat, &Wmat, &jac_work, &evals_d,
                            &resid_part, &resid_d, &flag, &HX, &diag0, &minratio, &rscratch, &occ_d, &Kc64, &Kcg,
                            &kshift, &pois_kb, &pois_m, &pois_work, &pois_q, &csel};
    for (chfsi::DevBuf *b : all) f(*b);
  }
};


namespace chfsi {

int fail(chfsi_ctx *c, int code, const std::string &msg);
int set_dev(chfsi_ctx *c);
int check_block(chfsi_ctx *c, const void *X, int64_t ld, int ncols);
int ensure_small(chfsi_ctx *c, int n);
// Workspace of one CholGS: device buffers for the overlap's split partials
// (part_elems doubles), S, the 32x32 diagonal inverses, Z and W (n x n each),
// the pivot diagnostics and the rotation's row panel (panel_elems doubles),
// and a host array of ceil(n/32) doubles for the pivot ratios.
struct CholWs {
  double *part = nullptr;
  size_t part_elems = 0;
  // complex blocks (interleaved re, im; ncols counts real columns): the raw
  // real Gram of the interleaved columns goes to G and its Hermitian
  // embedding to S (null for real blocks)
  double *G = nullptr;
  double *S = nullptr, *Z = nullptr, *W = nullptr, *dinv = nullptr, *diag0 = nullptr, *minratio = nullptr;
  int *flag = nullptr;
  double *panel = nullptr;
  size_t panel_elems = 0;
  double *host_ratio = nullptr;
};
int cholgs_core(chfsi_ctx *c, double *X, int64_t ld, int ncols, int mixed, double shift_rel, double *rmin,
                const CholWs &w);
// Looks up the device address of the allocation-free entry point's scratch
// array on `device` (current) once; 0 or an error status.
int noalloc_init(int device);
// the solve's CholGS (CholeskyQR2 / shifted Cholesky QR when needed); cplx:
// X is a complex block seen as interleaved reals (ld and nb count reals)
int orth_robust(chfsi_ctx *c, double *X, int64_t ld, int nb, int mixed, int *passes, bool cplx = false);
// Rayleigh-Ritz with HX in a caller buffer; evals/resid on the host
// Rayleigh-Ritz in three parts (a batch shares the middle one across problems)
int rr_project(chfsi_ctx *c, double *X, int64_t ld, int ncols, double *HX, int64_t ldh);
JacobiJob rr_eigen_job(chfsi_ctx *c, int ncols);
int rr_finish(chfsi_ctx *c, double *X, int64_t ld, int ncols, double *HX, int64_t ldh, double *evals,
              double *resid);
// Returns CHFSI_WARN_NOT_CONVERGED (with the results of the last Jacobi
// iterate) when the projected eigensolve ran out of sweeps.
int rr_impl(chfsi_ctx *c, double *X, int64_t ld, int ncols, double *HX, int64_t ldh, double *evals, double *resid,
            int *sweeps);
// Cells per work-group of the real cell kernel (tile width tw columns) for
// blocks of ncols columns: the context's setting, or (setting 0) the count
// among 1, 2, 4 that pads the fewest columns (ties: fewer cells); at least 16
// columns per cell either way.
int cells_per_tile(const chfsi_ctx *c, int ncols, int tw);
// Records the unconverged-eigensolve message and returns the warning.
int jacobi_warning(chfsi_ctx *c);
// Whether Rayleigh-Ritz obtains Htilde times the rotated columns by a fresh
// application (true) or by rotating HX (false), for ncols columns.
bool rr_reapply(const chfsi_ctx *c, int ncols);

}  // namespace chfsi

#define HIPCHK(ctx, call)                                                                         \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return chfsi::fail(ctx, e_ == hipErrorOutOfMemory ? CHFSI_ERR_OOM : CHFSI_ERR_HIP,          \
                         std::string(#call) + ": " + hipGetErrorString(e_));                      \
  } while (0)
