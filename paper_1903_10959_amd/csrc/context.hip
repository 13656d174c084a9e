// C ABI of the library: context, tables, and the host orchestration of the
// ChFSI steps (filter, CholGS, Rayleigh-Ritz, solve loop).  Every numerical
// step runs in the device kernels of hx.hip, dense.hip and small.hip; the host
// only computes scalars (recursion coefficients, bounds) and control flow.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/chfsi.h"
#include "ctx.hpp"
#include "kernels.hpp"
#include "mesh.hpp"

using namespace chfsi;

namespace {

// FP32 -> BF16 bits, round to nearest even (finite inputs)
static uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}
static float bf16_to_float(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

}  // namespace

namespace chfsi {
int fail(chfsi_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}



int set_dev(chfsi_ctx *c) {
  if (c->device < 0) return fail(c, CHFSI_ERR_STATE, "host-only context: no device work");
  HIPCHK(c, hipSetDevice(c->device));
  return 0;
}
}  // namespace chfsi

// ---------------------------------------------------------------------------
// lifetime
// ---------------------------------------------------------------------------
extern "C" int chfsi_create(chfsi_ctx **out, int device, void *hip_stream) {
  if (!out) return CHFSI_ERR_ARG;
  if (device != -1) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CHFSI_ERR_ARG;
  }
  if (device >= 0) {
    // the allocation-free CholGS needs its scratch array's address on this
    // device, looked up once per device with the device current
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return CHFSI_ERR_HIP;
    const int r = noalloc_init(device);
    if (hipSetDevice(prev) != hipSuccess) return CHFSI_ERR_HIP;
    if (r) return r;
  }
  chfsi_ctx *c = new (std::nothrow) chfsi_ctx();
  if (!c) return CHFSI_ERR_OOM;
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  const char *v = std::getenv("CHFSI_VERBOSE");
  c->verbose = v && v[0] && v[0] != '0';
  *out = c;
  return 0;
}

extern "C" int chfsi_destroy(chfsi_ctx *c) {
  if (!c) return CHFSI_ERR_ARG;
  if (c->device < 0) {
    delete c;
    return 0;
  }
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  c->each_buf([](DevBuf &b) { b.release(); });
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
  return 0;
}

extern "C" const char *chfsi_last_error(const chfsi_ctx *c) { return c ? c->err.c_str() : "null context"; }

extern "C" const char *chfsi_status_string(int s) {
  switch (s) {
    case CHFSI_OK: return "ok";
    case CHFSI_ERR_ARG: return "invalid argument";
    case CHFSI_ERR_STATE: return "mesh or potential not set";
    case CHFSI_ERR_OOM: return "device out of memory";
    case CHFSI_ERR_HIP: return "HIP runtime error";
    case CHFSI_ERR_NOT_SPD: return "overlap matrix not positive definite";
    case CHFSI_ERR_NONFINITE: return "non-finite values";
    case CHFSI_WARN_NOT_CONVERGED: return "not converged";
    default: return "unknown status";
  }
}

// ---------------------------------------------------------------------------
// setMesh / setPotential
// ---------------------------------------------------------------------------
static int upload_kpoint(chfsi_ctx *c);

static int set_mesh_impl(chfsi_ctx *c, double L, int n_el, int p, bool periodic) {
  if (!c) return CHFSI_ERR_ARG;
  if (c->device >= 0)
    if (int r = set_dev(c)) return r;
  MeshTables m;
  std::string msg = build_mesh(L, n_el, p, m, periodic);
  if (!msg.empty()) return fail(c, CHFSI_ERR_ARG, msg);
  c->has_mesh = c->has_pot = false;
  c->mesh = std::move(m);
  if (c->device < 0) {
    c->has_mesh = true;
    return 0;
  }
  const MeshTables &M = c->mesh;
  // the cell matrix, padded: np x np for the single-tile kernels (p <= 7);
  // np x npr, npr a whole number of 224-row groups, for the row-group kernel
  // of degrees 8..12
  const size_t nl = M.n_loc, np = M.np, npr = M.p > 7 ? (size_t)hx_rows_padded(M.n_loc) : np;
  HIPCHK(c, c->cmap.ensure(M.cmap.size() * sizeof(int32_t)));
  HIPCHK(c, c->cells.ensure(M.cell_order.size() * sizeof(int32_t)));
  HIPCHK(c, c->K64.ensure(np * npr * sizeof(double)));
  HIPCHK(c, c->K32.ensure(np * npr * sizeof(float)));
  HIPCHK(c, c->minv64.ensure(M.n_dof * sizeof(double)));
  HIPCHK(c, c->minv32.ensure(M.n_dof * sizeof(float)));
  std::vector<double> kp(np * npr, 0.0);
  std::vector<float> kp32(np * npr, 0.f);
  for (size_t i = 0; i < nl; ++i)
    for (size_t j = 0; j < nl; ++j) {
      kp[i * npr + j] = M.kcell[i * nl + j];
      kp32[i * npr + j] = (float)M.kcell[i * nl + j];
    }
  std::vector<double> mi(M.n_dof);
  std::vector<float> mi32(M.n_dof);
  for (int64_t i = 0; i < M.n_dof; ++i) {
    mi[i] = 1.0 / std::sqrt(M.mass[i]);
    mi32[i] = (float)mi[i];
  }
  HIPCHK(c, hipMemcpyAsync(c->cmap.p, M.cmap.data(), M.cmap.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->cells.p, M.cell_order.data(), M.cell_order.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->K64.p, kp.data(), kp.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->K32.p, kp32.data(), kp32.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->minv64.p, mi.data(), mi.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->minv32.p, mi32.data(), mi32.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  c->kc_stride = (int)npr;
  if (M.p > 7) {
    // no BF16 or complex cell kernel above p = 7
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->npb = 0;
    c->kvec[0] = c->kvec[1] = c->kvec[2] = 0.0;
    c->kin_k = 3.0 * c->mesh.lam1d_max;
    c->nk = 0;
    c->has_mesh = true;
    return 0;
  }
  // BF16 hi/lo split of the cell matrix, padded to a multiple of 32 (BF16 MFMA depth)
  c->npb = (int)((nl + 31) / 32 * 32);
  const size_t nb2 = (size_t)c->npb * c->npb;
  std::vector<uint16_t> kh(nb2, 0), kl(nb2, 0);
  for (size_t i = 0; i < nl; ++i)
    for (size_t j = 0; j < nl; ++j) {
      const float x = (float)M.kcell[i * nl + j];
      const uint16_t h = bf16_rne(x);
      kh[i * c->npb + j] = h;
      kl[i * c->npb + j] = bf16_rne(x - bf16_to_float(h));
    }
  HIPCHK(c, c->Kbh.ensure(nb2 * 2));
  HIPCHK(c, c->Kbl.ensure(nb2 * 2));
  HIPCHK(c, hipMemcpyAsync(c->Kbh.p, kh.data(), nb2 * 2, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->Kbl.p, kl.data(), nb2 * 2, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));  // host staging vectors go out of scope
  c->kvec[0] = c->kvec[1] = c->kvec[2] = 0.0;
  c->kin_k = 3.0 * c->mesh.lam1d_max;            // k = 0: the real periodic operator's bound
  c->nk = 0;                                     // a k-point group belongs to its mesh
  if (M.periodic)
    if (int r = upload_kpoint(c)) return r;
  c->has_mesh = true;
  return 0;
}

extern "C" int chfsi_set_mesh(chfsi_ctx *c, double L, int n_el, int p) { return set_mesh_impl(c, L, n_el, p, false); }

extern "C" int chfsi_set_mesh_periodic(chfsi_ctx *c, double L, int n_el, int p) {
  return set_mesh_impl(c, L, n_el, p, true);
}

// The complex cell matrix of Htilde_k as the real contraction operator of the
// interleaved layout: H^e = A - i B with A the stiffness of -1/2 Laplacian and
// B = k.G; for Y = H^e X with X = Xr + i Xi, Y_re = A Xr + B Xi and
// Y_im = A Xi - B Xr.  Stored as [A ; B^T] (2 np x np, row kappa holds the
// weights of contraction index kappa for every output row), so the second half
// of the contraction runs over the gathered X with its (re, im) pairs swapped
// and the imaginary outputs negated.
static int upload_kpoint(chfsi_ctx *c) {
  const MeshTables &M = c->mesh;
  const size_t nl = M.n_loc, np = M.np;
  std::vector<double> kc(2 * np * np, 0.0);
  for (size_t i = 0; i < nl; ++i)
    for (size_t j = 0; j < nl; ++j) {
      kc[i * np + j] = M.kcell[i * nl + j];
      const double b = c->kvec[0] * M.gcell[0][i * nl + j] + c->kvec[1] * M.gcell[1][i * nl + j] +
                       c->kvec[2] * M.gcell[2][i * nl + j];
      kc[(np + j) * np + i] = b;                   // B^T: row kappa = j, output i
    }
  HIPCHK(c, c->Kc64.ensure(kc.size() * sizeof(double)));
  HIPCHK(c, hipMemcpyAsync(c->Kc64.p, kc.data(), kc.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return 0;
}

extern "C" int chfsi_set_kpoint(chfsi_ctx *c, double kx, double ky, double kz) {
  if (!c) return CHFSI_ERR_ARG;
  if (!c->has_mesh || !c->mesh.periodic) return fail(c, CHFSI_ERR_STATE, "set_kpoint: needs a periodic mesh");
  if (c->mesh.p > 7) return fail(c, CHFSI_ERR_ARG, "set_kpoint: the complex cell kernel needs p <= 7");
  if (!std::isfinite(kx) || !std::isfinite(ky) || !std::isfinite(kz))
    return fail(c, CHFSI_ERR_ARG, "set_kpoint: k must be finite");
  c->kvec[0] = kx;
  c->kvec[1] = ky;
  c->kvec[2] = kz;
  // the kinetic part of the spectral bound at k (A_{-k} is the conjugate of A_k)
  double kin = 0;
  for (int d = 0; d < 3; ++d) {
    const double kd = std::fabs(c->kvec[d]);
    int same = -1;
    for (int e = 0; e < d; ++e)
      if (std::fabs(c->kvec[e]) == kd) same = e;
    kin += same >= 0 ? bloch_1d_max(c->mesh, std::fabs(c->kvec[same])) : bloch_1d_max(c->mesh, kd);
  }
  c->kin_k = kin;
  if (c->device < 0) return 0;
  if (int r = set_dev(c)) return r;
  return upload_kpoint(c);
}

extern "C" int chfsi_set_kpoints(chfsi_ctx *c, int nk, const double *k) {
  if (!c) return CHFSI_ERR_ARG;
  if (!c->has_mesh || !c->mesh.periodic) return fail(c, CHFSI_ERR_STATE, "set_kpoints: needs a periodic mesh");
  if (c->mesh.p > 7) return fail(c, CHFSI_ERR_ARG, "set_kpoints: the complex cell kernel needs p <= 7");
  if (nk < 1 || !k) return fail(c, CHFSI_ERR_ARG, "set_kpoints: need nk >= 1 and a host array of 3 nk values");
  for (int i = 0; i < 3 * nk; ++i)
    if (!std::isfinite(k[i])) return fail(c, CHFSI_ERR_ARG, "set_kpoints: k must be finite");
  c->kgroup.assign(k, k + 3 * nk);
  c->nk = nk;
  if (c->device < 0) return 0;
  if (int r = set_dev(c)) return r;
  const MeshTables &M = c->mesh;
  const size_t nl = M.n_loc, np = M.np, per = 2 * np * np;
  std::vector<double> kc(per * nk, 0.0), sh(nk);
  for (int g = 0; g < nk; ++g) {
    const double *kv = k + 3 * g;
    double *o = kc.data() + g * per;
    for (size_t i = 0; i < nl; ++i)
      for (size_t j = 0; j < nl; ++j) {
        o[i * np + j] = M.kcell[i * nl + j];
        o[(np + j) * np + i] =
            kv[0] * M.gcell[0][i * nl + j] + kv[1] * M.gcell[1][i * nl + j] + kv[2] * M.gcell[2][i * nl + j];
      }
    sh[g] = -0.5 * (kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2]);
  }
  HIPCHK(c, c->Kcg.ensure(kc.size() * sizeof(double)));
  HIPCHK(c, c->kshift.ensure(sh.size() * sizeof(double)));
  HIPCHK(c, hipMemcpyAsync(c->Kcg.p, kc.data(), kc.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->kshift.p, sh.data(), sh.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return 0;
}

extern "C" int chfsi_apply_complex_kpoints(chfsi_ctx *c, const void *X, void *Y, int64_t ld, int ncols,
                                           int64_t stride) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (!c->mesh.periodic || c->nk < 1)
    return fail(c, CHFSI_ERR_STATE, "apply_complex_kpoints: needs a periodic mesh and set_kpoints");
  const MeshTables &M = c->mesh;
  if (!Y || stride < M.n_dof * ld) return fail(c, CHFSI_ERR_ARG, "apply_complex_kpoints: stride < n_dof * ld");
  const char *xb = static_cast<const char *>(X), *yb = static_cast<const char *>(Y);
  const int64_t span = (int64_t)(c->nk - 1) * stride * 16 + M.n_dof * ld * 16;
  if (yb < xb + span && xb < yb + span) return fail(c, CHFSI_ERR_ARG, "apply_complex_kpoints: Y overlaps X");
  HxArgs<double> a;
  a.X = static_cast<const double *>(X);
  a.ldx = 2 * ld;
  a.Xp = nullptr;
  a.ldp = 0;
  a.Y = static_cast<double *>(Y);
  a.ldy = 2 * ld;
  a.K = c->Kcg.as<double>();
  a.cmap = c->cmap.as<int32_t>();
  a.n_loc = M.n_loc;
  a.np = M.np;
  a.q = M.q;
  a.n_el = M.n_el;
  a.cells = c->cells.as<int32_t>();
  a.minv = c->minv64.as<double>();
  a.V = c->V64.as<double>();
  a.ncols = 2 * ncols;
  a.s1 = 1.0;
  a.s2 = 0.0;
  a.shift = 0.0;
  a.variant = c->tile_variant;
  const CplxKpts g{c->nk, 2 * stride, 2 * stride, (int64_t)2 * M.np * M.np, c->kshift.as<double>()};
  for (int col = 0; col < 8; ++col)
    if (hx_cells_cplx_kpts_launch(a, g, M.color_offset[col], M.color_offset[col + 1], c->stream) != 0)
      return fail(c, CHFSI_ERR_ARG, "apply_complex_kpoints: unsupported cell size or grid too large");
  HIPCHK(c, hipGetLastError());
  return 0;
}

extern "C" int chfsi_apply_complex(chfsi_ctx *c, const void *X, void *Y, int64_t ld, int ncols) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (!c->mesh.periodic) return fail(c, CHFSI_ERR_STATE, "apply_complex: needs a periodic mesh");
  if (!Y || Y == X) return fail(c, CHFSI_ERR_ARG, "apply_complex: Y must be a separate device array");
  const MeshTables &M = c->mesh;
  HxArgs<double> a;
  a.X = static_cast<const double *>(X);
  a.ldx = 2 * ld;
  a.Xp = nullptr;
  a.ldp = 0;
  a.Y = static_cast<double *>(Y);
  a.ldy = 2 * ld;
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
  a.s1 = 1.0;
  a.s2 = 0.0;
  // V + |k|^2 / 2 on the diagonal: the epilogue adds s1 (V - shift) X
  a.shift = -0.5 * (c->kvec[0] * c->kvec[0] + c->kvec[1] * c->kvec[1] + c->kvec[2] * c->kvec[2]);
  a.variant = c->tile_variant;
  for (int col = 0; col < 8; ++col) {
    if (hx_cells_cplx_launch(a, M.color_offset[col], M.color_offset[col + 1], c->stream) != 0)
      return fail(c, CHFSI_ERR_ARG, "apply_complex: unsupported cell size");
  }
  HIPCHK(c, hipGetLastError());
  return 0;
}

extern "C" int chfsi_get_sizes(const chfsi_ctx *c, int64_t *n_dof, int64_t *n_cells, int *n_loc) {
  if (!c || !c->has_mesh) return CHFSI_ERR_STATE;
  if (n_dof) *n_dof = c->mesh.n_dof;
  if (n_cells) *n_cells = c->mesh.n_cells;
  if (n_loc) *n_loc = c->mesh.n_loc;
  return 0;
}

extern "C" int chfsi_get_cell_dof_map(const chfsi_ctx *c, int32_t *out) {
  if (!c || !c->has_mesh) return CHFSI_ERR_STATE;
  if (!out) return CHFSI_ERR_ARG;
  std::memcpy(out, c->mesh.cmap.data(), c->mesh.cmap.size() * sizeof(int32_t));
  return 0;
}

extern "C" int chfsi_get_cell_colors(const chfsi_ctx *c, uint8_t *out) {
  if (!c || !c->has_mesh) return CHFSI_ERR_STATE;
  if (!out) return CHFSI_ERR_ARG;
  std::memcpy(out, c->mesh.colors.data(), c->mesh.colors.size());
  return 0;
}

extern "C" int chfsi_get_dof_coords(const chfsi_ctx *c, double *xyz) {
  if (!c || !c->has_mesh) return CHFSI_ERR_STATE;
  if (!xyz) return CHFSI_ERR_ARG;
  dof_coords(c->mesh, xyz);
  return 0;
}

extern "C" int chfsi_get_mass(const chfsi_ctx *c, double *m) {
  if (!c || !c->has_mesh) return CHFSI_ERR_STATE;
  if (!m) return CHFSI_ERR_ARG;
  std::memcpy(m, c->mesh.mass.data(), c->mesh.mass.size() * sizeof(double));
  return 0;
}

extern "C" int chfsi_get_cell_matrix(const chfsi_ctx *c, double *k) {
  if (!c || !c->has_mesh) return CHFSI_ERR_STATE;
  if (!k) return CHFSI_ERR_ARG;
  std::memcpy(k, c->mesh.kcell.data(), c->mesh.kcell.size() * sizeof(double));
  return 0;
}

extern "C" int chfsi_set_potential(chfsi_ctx *c, const double *v, int64_t n_dof, int v_on_device) {
  if (!c) return CHFSI_ERR_ARG;
  if (!c->has_mesh) return fail(c, CHFSI_ERR_STATE, "set_potential before set_mesh");
  if (!v || n_dof != c->mesh.n_dof) return fail(c, CHFSI_ERR_ARG, "set_potential: size mismatch or null");
  if (c->device < 0 && v_on_device) return fail(c, CHFSI_ERR_ARG, "host-only context takes a host potential");
  if (c->device >= 0)
    if (int r = set_dev(c)) return r;
  std::vector<double> hv(n_dof);
  if (v_on_device) {
    HIPCHK(c, hipMemcpyAsync(hv.data(), v, n_dof * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  else std::memcpy(hv.data(), v, n_dof * sizeof(double));
  double vmax = -INFINITY;
  for (int64_t i = 0; i < n_dof; ++i) {
    if (!std::isfinite(hv[i])) return fail(c, CHFSI_ERR_ARG, "set_potential: non-finite value");
    vmax = std::max(vmax, hv[i]);
  }
  c->vmax = vmax;
  c->ub = 3.0 * c->mesh.lam1d_max + vmax;
  if (c->device < 0) {
    c->has_pot = true;
    return 0;
  }
  std::vector<float> hv32(n_dof);
  for (int64_t i = 0; i < n_dof; ++i) hv32[i] = (float)hv[i];
  HIPCHK(c, c->V64.ensure(n_dof * sizeof(double)));
  HIPCHK(c, c->V32.ensure(n_dof * sizeof(float)));
  HIPCHK(c, hipMemcpyAsync(c->V64.p, hv.data(), n_dof * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->V32.p, hv32.data(), n_dof * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->vmax = vmax;
  c->ub = 3.0 * c->mesh.lam1d_max + vmax;
  c->has_pot = true;
  return 0;
}

extern "C" int chfsi_get_upper_bound(const chfsi_ctx *c, double *b) {
  if (!c || !c->has_pot) return CHFSI_ERR_STATE;
  if (!b) return CHFSI_ERR_ARG;
  *b = c->ub;
  return 0;
}

extern "C" int chfsi_get_upper_bound_k(const chfsi_ctx *c, double *b) {
  if (!c || !c->has_pot || !c->mesh.periodic) return CHFSI_ERR_STATE;
  if (!b) return CHFSI_ERR_ARG;
  *b = c->kin_k + c->vmax;
  return 0;
}

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------
extern "C" int chfsi_set_timing(chfsi_ctx *c, int enable) {
  if (!c) return CHFSI_ERR_ARG;
  c->timing = enable != 0;
  return 0;
}

int chfsi::cells_per_tile(const chfsi_ctx *c, int ncols, int tw) {
  // at least 16 columns per cell; one cell per tile above p = 6
  const int max_cpt = c->mesh.p > 6 ? 1 : (tw >= 64 ? 4 : (tw >= 32 ? 2 : 1));
  if (c->cpt_setting > 0) return std::min(c->cpt_setting, max_cpt);
  int best = 1;
  int64_t best_pad = -1;
  for (int cpt = 1; cpt <= max_cpt; cpt *= 2) {
    const int cw = tw / cpt;
    const int64_t pad = (int64_t)(ncols + cw - 1) / cw * cw - ncols;
    if (best_pad < 0 || pad < best_pad) {
      best = cpt;
      best_pad = pad;
    }
  }
  return best;
}

extern "C" int chfsi_set_cells_per_tile(chfsi_ctx *c, int cpt) {
  if (!c) return CHFSI_ERR_ARG;
  if (cpt != 0 && cpt != 1 && cpt != 2 && cpt != 4) return fail(c, CHFSI_ERR_ARG, "cells per tile must be 0, 1, 2 or 4");
  c->cpt_setting = cpt;
  return 0;
}

extern "C" int chfsi_set_tile_variant(chfsi_ctx *c, int variant) {
  if (!c) return CHFSI_ERR_ARG;
  if (variant < -1 || variant > 1) return fail(c, CHFSI_ERR_ARG, "tile variant must be -1, 0 or 1");
  c->tile_variant = variant;
  return 0;
}

extern "C" int chfsi_set_jacobi_sweeps(chfsi_ctx *c, int max_sweeps) {
  if (!c) return CHFSI_ERR_ARG;
  if (max_sweeps < 1 || max_sweeps > 1000) return fail(c, CHFSI_ERR_ARG, "Jacobi sweeps must be in 1..1000");
  c->jac_sweeps = max_sweeps;
  return 0;
}

extern "C" int chfsi_set_rr_residual(chfsi_ctx *c, int mode) {
  if (!c) return CHFSI_ERR_ARG;
  if (mode < 0 || mode > 2) return fail(c, CHFSI_ERR_ARG, "rr residual mode must be 0, 1 or 2");
  c->rr_residual = mode;
  return 0;
}

extern "C" int chfsi_reset_timing(chfsi_ctx *c) {
  if (!c) return CHFSI_ERR_ARG;
  c->ev_used = 0;
  c->cell_vecs = 0;
  return 0;
}

extern "C" int chfsi_last_filter_timing(chfsi_ctx *c, double *ms_cells, int *n_launches, int64_t *cell_vecs) {
  if (!c) return CHFSI_ERR_ARG;
  if (int r = set_dev(c)) return r;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double tot = 0;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[i], c->ev_pool[i + 1]));
    tot += ms;
  }
  if (ms_cells) *ms_cells = tot;
  if (n_launches) *n_launches = (int)(c->ev_used / 2);
  if (cell_vecs) *cell_vecs = c->cell_vecs;
  return 0;
}

static hipEvent_t next_event(chfsi_ctx *c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// ---------------------------------------------------------------------------
// Htilde-based step on one column block, any working precision T
// ---------------------------------------------------------------------------
// bf: 0 = products in T; 1 = BF16 inputs (T = float); 2 = BF16 hi/lo split (T = float)
template <typename T>
static int cheb_step_t(chfsi_ctx *c, const T *X, int64_t ldx, const T *Xp, int64_t ldp, T *Y, int64_t ldy,
                       int ncols, double s1, double s2, double shift, int bf = 0) {
  const MeshTables &M = c->mesh;
  const T *V = std::is_same<T, double>::value ? (const T *)c->V64.p : (const T *)c->V32.p;
  const T *K = std::is_same<T, double>::value ? (const T *)c->K64.p : (const T *)c->K32.p;
  const T *mi = std::is_same<T, double>::value ? (const T *)c->minv64.p : (const T *)c->minv32.p;
  HxArgs<T> a;
  a.X = X;
  a.ldx = ldx;
  a.Xp = Xp;
  a.ldp = ldp;
  a.Y = Y;
  a.ldy = ldy;
  a.K = K;
  a.cmap = c->cmap.as<int32_t>();
  a.n_loc = M.n_loc;
  a.np = M.np;
  a.q = M.q;
  a.n_el = M.n_el;
  a.cells = c->cells.as<int32_t>();
  a.minv = mi;
  a.V = V;
  a.ncols = ncols;
  a.s1 = (T)s1;
  a.s2 = (T)s2;
  a.shift = (T)shift;
  a.variant = c->tile_variant;
  a.cpt = cells_per_tile(c, ncols, hx_tile_width<T>(M.np, c->tile_variant, 1));
  for (int col = 0; col < 8; ++col) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
      e0 = next_event(c);
      if (e0) (void)hipEventRecord(e0, c->stream);
    }
    int lr;
    if (M.p > 7) {
      lr = bf ? -1 : hx_rows_launch<T>(a, c->kc_stride, M.color_offset[col], M.color_offset[col + 1], c->stream);
    } else if (bf) {
      HxBf16Args b;
      b.X = (const float *)X;
      b.ldx = ldx;
      b.Xp = (const float *)Xp;
      b.ldp = ldp;
      b.Y = (float *)Y;
      b.ldy = ldy;
      b.Kh = c->Kbh.as<const __bf16>();
      b.Kl = c->Kbl.as<const __bf16>();
      b.cmap = a.cmap;
      b.n_loc = M.n_loc;
      b.npb = c->npb;
      b.q = M.q;
      b.n_el = M.n_el;
      b.cells = a.cells;
      b.minv = c->minv32.as<float>();
      b.V = c->V32.as<float>();
      b.ncols = ncols;
      b.s1 = (float)s1;
      b.s2 = (float)s2;
      b.shift = (float)shift;
      b.split = bf == 2;
      b.cbw = c->tile_variant == 1 ? 1 : 2;
      lr = hx_cells_bf16_launch(b, M.color_offset[col], M.color_offset[col + 1], c->stream);
    } else {
      lr = hx_cells_launch<T>(a, M.color_offset[col], M.color_offset[col + 1], c->stream);
    }
    if (lr != 0)
      return fail(c, CHFSI_ERR_ARG, bf ? "no BF16 cell kernel for this degree (p <= 7)" : "no cell kernel for this degree");
    if (c->timing && e0) {
      e1 = next_event(c);
      if (e1) (void)hipEventRecord(e1, c->stream);
    }
  }
  if (c->timing) c->cell_vecs += (int64_t)M.n_cells * ncols;   // the work of the timed launches
  HIPCHK(c, hipGetLastError());
  return 0;
}

int chfsi::check_block(chfsi_ctx *c, const void *X, int64_t ld, int ncols) {
  if (!c) return CHFSI_ERR_ARG;
  if (c->device < 0) return fail(c, CHFSI_ERR_STATE, "host-only context: no device work");
  if (!c->has_mesh || !c->has_pot) return fail(c, CHFSI_ERR_STATE, "mesh and potential must be set first");
  if (!X || ncols < 1 || ld < ncols) return fail(c, CHFSI_ERR_ARG, "bad block arguments (pointer, ncols, ld)");
  return set_dev(c);
}

extern "C" int chfsi_cheb_step(chfsi_ctx *c, const double *X, const double *Xp, double *Y, int64_t ld, int ncols,
                               double s1, double s2, double shift) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (!Y || Y == X || (Xp && Y == Xp)) return fail(c, CHFSI_ERR_ARG, "cheb_step: Y must not alias X or Xprev");
  return cheb_step_t<double>(c, X, ld, Xp, ld, Y, ld, ncols, s1, s2, shift);
}

// FP32 copies of a column block live in fbuf[] (ld = width)
static int ensure_fbufs(chfsi_ctx *c, size_t elem, int width) {
  const size_t bytes = (size_t)c->mesh.n_dof * width * elem;
  for (int i = 0; i < 3; ++i) HIPCHK(c, c->fbuf[i].ensure(bytes));
  return 0;
}

extern "C" int chfsi_apply(chfsi_ctx *c, const double *X, double *Y, int64_t ld, int ncols, chfsi_prec prec) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (!Y || X == Y) return fail(c, CHFSI_ERR_ARG, "apply: Y must not alias X");
  if (prec == CHFSI_FP64) return cheb_step_t<double>(c, X, ld, nullptr, 0, Y, ld, ncols, 1.0, 0.0, 0.0);
  if (prec != CHFSI_FP32 && prec != CHFSI_BF16 && prec != CHFSI_BF16X3)
    return fail(c, CHFSI_ERR_ARG, "apply: unknown precision");
  const int bf = prec == CHFSI_BF16 ? 1 : (prec == CHFSI_BF16X3 ? 2 : 0);
  const int64_t nd = c->mesh.n_dof;
  const int bw = std::min(ncols, 256);
  if (int r = ensure_fbufs(c, sizeof(float), bw)) return r;
  for (int j0 = 0; j0 < ncols; j0 += bw) {
    const int w = std::min(bw, ncols - j0);
    float *a = c->fbuf[0].as<float>(), *b = c->fbuf[1].as<float>();
    copy_cols_launch<double, float>(X + j0, ld, a, w, nd, w, c->stream);
    if (int r = cheb_step_t<float>(c, a, w, nullptr, 0, b, w, w, 1.0, 0.0, 0.0, bf)) return r;
    copy_cols_launch<float, double>(b, w, Y + j0, ld, nd, w, c->stream);
  }
  HIPCHK(c, hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------------------
// chebyshevFilter
// ---------------------------------------------------------------------------
template <typename T>
static int filter_block(chfsi_ctx *c, T *z0, int64_t ld0, T *w1, T *w2, int64_t ldw, int ncols, int degree,
                        double a, double b, double a0, int bf = 0) {
  // normalised recursion: rho_1 = 1/xi0, rho_{k+1} = 1/(2 xi0 - rho_k);
  // Z_1 = (rho_1/e)(H - c) Z_0;  Z_{k+1} = (2 rho_{k+1}/e)(H - c) Z_k - rho_{k+1} rho_k Z_{k-1}
  const double cc = 0.5 * (a + b), e = 0.5 * (b - a), xi0 = (a0 - cc) / e;
  T *buf[3] = {z0, w1, w2};
  const int64_t lds[3] = {ld0, ldw, ldw};
  int cur = 0, prev = -1;
  double rho = 1.0 / xi0;
  for (int k = 0; k < degree; ++k) {
    double s1, s2;
    if (k == 0) {
      s1 = rho / e;
      s2 = 0.0;
    } else {
      double rn = 1.0 / (2.0 * xi0 - rho);
      s1 = 2.0 * rn / e;
      s2 = -rn * rho;
      rho = rn;
    }
    int out = 0;
    while (out == cur || out == prev) ++out;
    if (int r = cheb_step_t<T>(c, buf[cur], lds[cur], prev >= 0 ? buf[prev] : nullptr, prev >= 0 ? lds[prev] : 0,
                               buf[out], lds[out], ncols, s1, s2, cc, bf))
      return r;
    prev = cur;
    cur = out;
  }
  if (cur != 0) copy_cols_launch<T, T>(buf[cur], lds[cur], z0, ld0, c->mesh.n_dof, ncols, c->stream);
  return 0;
}

extern "C" int chfsi_chebyshev_filter(chfsi_ctx *c, double *X, int64_t ld, int ncols, int degree, double a,
                                      double b, double a0, chfsi_prec prec, int block_width) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (degree < 0 || !(a0 < a) || !(a < b)) return fail(c, CHFSI_ERR_ARG, "filter: need a0 < a < b, degree >= 0");
  if (prec != CHFSI_FP64 && prec != CHFSI_FP32 && prec != CHFSI_BF16 && prec != CHFSI_BF16X3)
    return fail(c, CHFSI_ERR_ARG, "filter: unknown precision");
  const int bf = prec == CHFSI_BF16 ? 1 : (prec == CHFSI_BF16X3 ? 2 : 0);
  if (degree == 0) return 0;
  const int64_t nd = c->mesh.n_dof;
  int bw = block_width > 0 ? block_width : 128;
  bw = std::min(bw, ncols);
  if (prec == CHFSI_FP64) {
    if (int r = ensure_fbufs(c, sizeof(double), bw)) return r;
    for (int j0 = 0; j0 < ncols; j0 += bw) {
      const int w = std::min(bw, ncols - j0);
      if (int r = filter_block<double>(c, X + j0, ld, c->fbuf[1].as<double>(), c->fbuf[2].as<double>(), w, w,
                                       degree, a, b, a0))
        return r;
    }
  } else {
    if (int r = ensure_fbufs(c, sizeof(float), bw)) return r;
    for (int j0 = 0; j0 < ncols; j0 += bw) {
      const int w = std::min(bw, ncols - j0);
      float *f0 = c->fbuf[0].as<float>();
      copy_cols_launch<double, float>(X + j0, ld, f0, w, nd, w, c->stream);
      if (int r = filter_block<float>(c, f0, w, c->fbuf[1].as<float>(), c->fbuf[2].as<float>(), w, w, degree, a,
                                      b, a0, bf))
        return r;
      copy_cols_launch<float, double>(f0, w, X + j0, ld, nd, w, c->stream);
    }
  }
  HIPCHK(c, c->flag.ensure(4 * sizeof(int)));
  zero_int_launch(c->flag.as<int>(), 1, c->stream);
  nonfinite_launch<double>(X, ld, nd, ncols, c->flag.as<int>(), c->stream);
  int hflag = 0;
  HIPCHK(c, hipMemcpyAsync(&hflag, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (hflag) return fail(c, CHFSI_ERR_NONFINITE, "filter produced NaN/Inf (upper bound below lambda_max?)");
  return 0;
}

// ---------------------------------------------------------------------------
// orthonormalize (CholGS)
// ---------------------------------------------------------------------------
int chfsi::ensure_small(chfsi_ctx *c, int n) {
  const size_t nn = (size_t)n * n;
  const int nb = (n + 31) / 32;
  HIPCHK(c, c->Smat.ensure(nn * sizeof(double)));
  HIPCHK(c, c->dinv.ensure((size_t)nb * 32 * 32 * sizeof(double)));
  HIPCHK(c, c->Zmat.ensure(nn * sizeof(double)));
  HIPCHK(c, c->Wmat.ensure(nn * sizeof(double)));
  HIPCHK(c, c->jac_work.ensure(jacobi_work_elems(n) * sizeof(double)));
  HIPCHK(c, c->evals_d.ensure((size_t)n * sizeof(double)));
  HIPCHK(c, c->resid_d.ensure((size_t)n * sizeof(double)));
  HIPCHK(c, c->flag.ensure(4 * sizeof(int)));
  HIPCHK(c, c->diag0.ensure((size_t)n * sizeof(double)));
  HIPCHK(c, c->minratio.ensure((size_t)nb * sizeof(double)));
  HIPCHK(c, c->rscratch.ensure(rmul_scratch_elems(c->mesh.n_dof, n) * sizeof(double)));
  const size_t hs = std::max((size_t)nb + 16, jacobi_norms_elems(1));
  if (c->host_scratch.size() < hs) c->host_scratch.resize(hs);
  HIPCHK(c, c->gram_part.ensure(gram_part_elems(c->mesh.n_dof, n) * sizeof(double)));
  HIPCHK(c, c->resid_part.ensure((size_t)resid_nchunk(c->mesh.n_dof) * n * sizeof(double)));
  return 0;
}

// CholGS on X (Alg. 3) with the workspace w.  shift_rel > 0 factors
// S + shift_rel * max(diag S) I (shifted Cholesky QR).  *rmin receives
// min_j d_j / S_jj over the pivots.
int chfsi::cholgs_core(chfsi_ctx *c, double *X, int64_t ld, int ncols, int mixed, double shift_rel, double *rmin,
                       const CholWs &w) {
  const int64_t nd = c->mesh.n_dof;
  const int nb32 = (ncols + 31) / 32;
  if (gram_launch_capped(X, ld, X, ld, nd, ncols, w.part, w.part_elems, w.G ? w.G : w.S, mixed ? 1 : 0,
                         c->stream) != 0)
    return fail(c, CHFSI_ERR_ARG, "orthonormalize: overlap workspace too small");
  if (w.G) herm_embed_launch(w.G, ncols, w.S, c->stream);   // complex: S = emb(X^H X)
  zero_int_launch(w.flag, 1, c->stream);
  potrf_launch(w.S, ncols, w.dinv, w.flag, w.diag0, w.minratio, shift_rel, c->stream);
  int hflag = 0;
  HIPCHK(c, hipMemcpyAsync(&hflag, w.flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(w.host_ratio, w.minratio, nb32 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double m = 1.0;
  for (int i = 0; i < nb32; ++i) m = std::min(m, w.host_ratio[i]);
  if (rmin) *rmin = m;
  if (hflag) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "CholGS: overlap not numerically positive definite (pivot %d, ratio %.3g)",
                  hflag - 1, m);
    return fail(c, CHFSI_ERR_NOT_SPD, msg);
  }
  trtri_t_launch(w.S, w.dinv, ncols, w.Z, w.W, c->stream);
  if (rmul_launch(X, ld, nd, ncols, w.W, 1, mixed ? 1 : 0, w.panel, w.panel_elems, c->stream) != 0)
    return fail(c, CHFSI_ERR_ARG, "orthonormalize: block too wide for the row-panel kernel");
  HIPCHK(c, hipGetLastError());
  return 0;
}

// CholGS with the context's own (grown on demand) workspace; cplx: X is a
// complex block as interleaved reals (ld, ncols count reals).
static int cholgs_impl(chfsi_ctx *c, double *X, int64_t ld, int ncols, int mixed, double shift_rel, double *rmin,
                       bool cplx = false) {
  if (int r = ensure_small(c, ncols)) return r;
  CholWs w;
  if (cplx) w.G = c->Zmat.as<double>();     // consumed before the inverse uses Z
  w.part = c->gram_part.as<double>();
  w.part_elems = c->gram_part.bytes / sizeof(double);
  w.S = c->Smat.as<double>();
  w.Z = c->Zmat.as<double>();
  w.W = c->Wmat.as<double>();
  w.dinv = c->dinv.as<double>();
  w.diag0 = c->diag0.as<double>();
  w.minratio = c->minratio.as<double>();
  w.flag = c->flag.as<int>();
  w.panel = c->rscratch.as<double>();
  w.panel_elems = c->rscratch.bytes / sizeof(double);
  w.host_ratio = c->host_scratch.data();
  return cholgs_core(c, X, ld, ncols, mixed, shift_rel, rmin, w);
}

extern "C" int chfsi_orthonormalize(chfsi_ctx *c, double *X, int64_t ld, int ncols, int mixed) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  return cholgs_impl(c, X, ld, ncols, mixed, 0.0, nullptr);
}

// The solve's orthonormalisation: CholGS, repeated while the smallest relative
// pivot shows lost orthogonality (CholeskyQR2), with the shifted Cholesky QR
// of Fukaya et al. when the overlap is numerically singular.
int chfsi::orth_robust(chfsi_ctx *c, double *X, int64_t ld, int nb, int mixed, int *passes, bool cplx) {
  double rmin = 1.0;
  int np = 1;
  int st = cholgs_impl(c, X, ld, nb, mixed, 0.0, &rmin, cplx);
  if (st == CHFSI_ERR_NOT_SPD) {
    const double u = 1.1102230246251565e-16;
    const double m = (double)c->mesh.n_dof, n = nb;
    const double shift_rel = 11.0 * (m * n + n * (n + 1.0)) * u * n;
    st = cholgs_impl(c, X, ld, nb, mixed, shift_rel, &rmin, cplx);
    rmin = 0.0;
    ++np;
  }
  if (st) return st;
  for (int k = 0; k < 3 && rmin < 1e-2; ++k) {
    st = cholgs_impl(c, X, ld, nb, mixed, 0.0, &rmin, cplx);
    ++np;
    if (st) return st;
  }
  if (passes) *passes = np;
  return 0;
}

// ---------------------------------------------------------------------------
// rayleighRitz
// ---------------------------------------------------------------------------
// Part 1: HX = Htilde X and the projected Hamiltonian G = X^T HX (into Smat).
int chfsi::rr_project(chfsi_ctx *c, double *X, int64_t ld, int ncols, double *HX, int64_t ldh) {
  const int64_t nd = c->mesh.n_dof;
  if (int r = cheb_step_t<double>(c, X, ld, nullptr, 0, HX, ldh, ncols, 1.0, 0.0, 0.0)) return r;
  gram_launch(X, ld, HX, ldh, nd, ncols, c->gram_part.as<double>(), c->Smat.as<double>(), 0, c->stream);
  return 0;
}

// The eigensolve of part 2 as a job of the (batched) Jacobi driver: G in
// Smat, eigenvectors into Wmat, eigenvalues into evals_d.
chfsi::JacobiJob chfsi::rr_eigen_job(chfsi_ctx *c, int ncols) {
  return JacobiJob{c->Smat.as<double>(), ncols, c->jac_work.as<double>(), c->evals_d.as<double>(),
                   c->Wmat.as<double>()};
}

// The residuals of k rotated columns need Htilde applied to them: either HX is
// rotated with X (2 n_dof ncols flops per column, a plain GEMM) or Htilde is
// applied again (the cell products, 2 n_cells np^2 flops per column, which run
// at a lower fraction of peak than the GEMM: weighted 1.4).  Both give Htilde
// times the rotated columns; the cheaper is taken unless the mode forces one.
bool chfsi::rr_reapply(const chfsi_ctx *c, int ncols) {
  if (c->rr_residual != 0) return c->rr_residual == 2;
  const MeshTables &M = c->mesh;
  const double cells = (double)M.n_el * M.n_el * M.n_el;
  return 1.4 * cells * M.np * M.np < (double)M.n_dof * ncols;
}

// Rotates X by W (ncols x nout, row stride ncols): in place into the columns
// [col0, col0 + nout) of X, or into Xout (ldo) when given, leaving X as it is.
// HX[:, col0 : col0 + nout] then holds Htilde times the rotated columns, by
// rotation or by a fresh application.
static int rr_rotate(chfsi_ctx *c, double *X, int64_t ld, int ncols, double *HX, int64_t ldh, const double *W,
                     int nout, int col0, double *Xout = nullptr, int64_t ldo = 0) {
  const int64_t nd = c->mesh.n_dof;
  double *scr = c->rscratch.as<double>();
  const size_t se = c->rscratch.bytes / sizeof(double);
  const int st = Xout ? rmul_out_launch(X, ld, nd, ncols, W, ncols, nout, Xout, ldo, c->stream)
                      : rmul_cols_launch(X, ld, nd, ncols, W, ncols, nout, col0, 0, 0, scr, se, c->stream);
  if (st != 0) return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz: block too wide for the row-panel kernel");
  if (rr_reapply(c, ncols))
    return cheb_step_t<double>(c, Xout ? Xout : X + col0, Xout ? ldo : ld, nullptr, 0, HX + col0, ldh, nout, 1.0,
                               0.0, 0.0);
  if (rmul_cols_launch(HX, ldh, nd, ncols, W, ncols, nout, col0, 0, 0, scr, se, c->stream) != 0)
    return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz: block too wide for the row-panel kernel");
  return 0;
}

int chfsi::jacobi_warning(chfsi_ctx *c) {
  char msg[128];
  std::snprintf(msg, sizeof msg, "Rayleigh-Ritz: the projected eigensolve did not converge in %d Jacobi sweeps",
                c->jac_sweeps);
  return fail(c, CHFSI_WARN_NOT_CONVERGED, msg);
}

// Part 3: X <- X Q, HX = Htilde X (rr_rotate), residual norms; evals and
// resid to the host.
int chfsi::rr_finish(chfsi_ctx *c, double *X, int64_t ld, int ncols, double *HX, int64_t ldh, double *evals,
                     double *resid) {
  const int64_t nd = c->mesh.n_dof;
  if (int r = rr_rotate(c, X, ld, ncols, HX, ldh, c->Wmat.as<double>(), ncols, 0)) return r;
  resid_launch(X, ld, HX, ldh, c->evals_d.as<double>(), nd, ncols, c->resid_part.as<double>(),
               c->resid_d.as<double>(), c->stream);
  HIPCHK(c, hipMemcpyAsync(evals, c->evals_d.p, ncols * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(resid, c->resid_d.p, ncols * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipGetLastError());
  return 0;
}

int chfsi::rr_impl(chfsi_ctx *c, double *X, int64_t ld, int ncols, double *HX, int64_t ldh, double *evals,
                   double *resid, int *sweeps) {
  if (int r = rr_project(c, X, ld, ncols, HX, ldh)) return r;
  const JacobiJob job = rr_eigen_job(c, ncols);
  const int jr = jacobi_eigh(job.A, ncols, job.work, job.evals, job.Q, 1e-14, c->jac_sweeps, c->host_scratch.data(),
                             c->stream, sweeps);
  if (jr < 0) return fail(c, CHFSI_ERR_HIP, "Jacobi eigensolver: HIP error");
  if (int r = rr_finish(c, X, ld, ncols, HX, ldh, evals, resid)) return r;
  return jr > 0 ? jacobi_warning(c) : 0;
}

extern "C" int chfsi_rayleigh_ritz(chfsi_ctx *c, double *X, int64_t ld, int ncols, double *evals, double *resid,
                                   double *HX_out) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (!evals || !resid) return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz: evals/resid must be host arrays");
  if (int r = ensure_small(c, ncols)) return r;
  double *HX = HX_out;
  int64_t ldh = ld;
  if (!HX) {
    HIPCHK(c, c->HX.ensure((size_t)c->mesh.n_dof * ncols * sizeof(double)));
    HX = c->HX.as<double>();
    ldh = ncols;
  }
  if (HX == X) return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz: HX_out must not alias X");
  return rr_impl(c, X, ld, ncols, HX, ldh, evals, resid, nullptr);
}

// ---------------------------------------------------------------------------
// rayleighRitz with spectrum splitting (Alg. 4) and the mixed-precision
// projected Hamiltonian
// ---------------------------------------------------------------------------
extern "C" int chfsi_rayleigh_ritz_split(chfsi_ctx *c, double *X, int64_t ld, int ncols, int n_fr, int mixed,
                                         double *Xfr, int64_t ldfr, double *evals_fr, double *resid_fr) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (n_fr < 1 || n_fr > ncols) return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz_split: n_fr must be in 1..ncols");
  if (!evals_fr || !resid_fr) return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz_split: evals/resid must be host arrays");
  if (Xfr) {
    if (ldfr < n_fr) return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz_split: ldfr < n_fr");
    const double *xe = X + (c->mesh.n_dof - 1) * ld + ncols;
    const double *fe = Xfr + (c->mesh.n_dof - 1) * ldfr + n_fr;
    if (Xfr < xe && X < fe) return fail(c, CHFSI_ERR_ARG, "rayleigh_ritz_split: Xfr overlaps X");
  }
  if (int r = ensure_small(c, ncols)) return r;
  const int64_t nd = c->mesh.n_dof;
  HIPCHK(c, c->HX.ensure((size_t)nd * ncols * sizeof(double)));
  double *HX = c->HX.as<double>();
  const int64_t ldh = ncols;
  const int n_oc = ncols - n_fr;
  // step 1: Hhat = X^T Htilde X; mixed: the fr-fr block in FP64, the rest FP32
  if (int r = cheb_step_t<double>(c, X, ld, nullptr, 0, HX, ldh, ncols, 1.0, 0.0, 0.0)) return r;
  double *G = c->Smat.as<double>();
  if (mixed)
    gram_split_launch(X, ld, HX, ldh, nd, ncols, c->gram_part.as<double>(), G, n_oc, c->stream);
  else
    gram_launch(X, ld, HX, ldh, nd, ncols, c->gram_part.as<double>(), G, 0, c->stream);
  // step 2: eigenpairs of Hhat (all of them; the N_fr largest are used)
  const JacobiJob job = rr_eigen_job(c, ncols);
  const int jr = jacobi_eigh(job.A, ncols, job.work, job.evals, job.Q, 1e-14, c->jac_sweeps, c->host_scratch.data(),
                             c->stream, nullptr);
  if (jr < 0) return fail(c, CHFSI_ERR_HIP, "Jacobi eigensolver: HIP error");
  // step 3: partial rotation X Q_fr, into Xfr or over the trailing N_fr
  // columns of X (and Htilde on the rotated columns, for their residuals)
  if (int r = rr_rotate(c, X, ld, ncols, HX, ldh, job.Q + n_oc, n_fr, n_oc, Xfr, ldfr)) return r;
  resid_launch(Xfr ? Xfr : X + n_oc, Xfr ? ldfr : ld, HX + n_oc, ldh, job.evals + n_oc, nd, n_fr,
               c->resid_part.as<double>(), c->resid_d.as<double>(), c->stream);
  HIPCHK(c, hipMemcpyAsync(evals_fr, job.evals + n_oc, n_fr * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(resid_fr, c->resid_d.p, n_fr * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipGetLastError());
  return jr > 0 ? jacobi_warning(c) : 0;
}

// ---------------------------------------------------------------------------
// Electron density (Alg. 5)
// ---------------------------------------------------------------------------
// Fermi-Dirac occupancy (Sec. 2.1); exp overflows to +inf for large
// arguments, giving 0, which is the limit.
static double fermi_dirac(double e, double mu, double sigma) { return 1.0 / (1.0 + std::exp((e - mu) / sigma)); }

static double electron_count(const double *e, int n, int n_oc, double mu, double sigma) {
  double s = 0;
  for (int k = 0; k < n; ++k) s += fermi_dirac(e[k], mu, sigma);
  return 2.0 * (n_oc + s);
}

extern "C" int chfsi_fermi_level(const double *evals_fr, int n_fr, int n_oc, double n_electrons, double sigma,
                                 double *mu) {
  if (!evals_fr || !mu || n_fr < 1 || n_oc < 0 || !(sigma > 0) || !std::isfinite(sigma)) return CHFSI_ERR_ARG;
  if (!(n_electrons > 2.0 * n_oc && n_electrons < 2.0 * (n_oc + n_fr))) return CHFSI_ERR_ARG;
  double lo = evals_fr[0], hi = evals_fr[0];
  for (int k = 0; k < n_fr; ++k) {
    if (!std::isfinite(evals_fr[k])) return CHFSI_ERR_ARG;
    lo = std::min(lo, evals_fr[k]);
    hi = std::max(hi, evals_fr[k]);
  }
  // bracket: the count rises monotonically in mu from 2 n_oc to 2 (n_oc + n_fr)
  for (double step = 40.0 * sigma + (hi - lo); electron_count(evals_fr, n_fr, n_oc, lo, sigma) >= n_electrons;
       step *= 2)
    lo -= step;
  for (double step = 40.0 * sigma + (hi - lo); electron_count(evals_fr, n_fr, n_oc, hi, sigma) <= n_electrons;
       step *= 2)
    hi += step;
  // bisection to the last representable midpoint
  for (int it = 0; it < 2000; ++it) {
    const double m = lo + 0.5 * (hi - lo);
    if (m <= lo || m >= hi) break;
    if (electron_count(evals_fr, n_fr, n_oc, m, sigma) < n_electrons) lo = m;
    else hi = m;
  }
  *mu = lo + 0.5 * (hi - lo);
  return 0;
}

extern "C" int chfsi_density(chfsi_ctx *c, const double *X, int64_t ld, int ncols, const double *Xfr, int64_t ldfr,
                             int n_fr, const double *evals_fr, double mu, double sigma, double *rho) {
  if (!c) return CHFSI_ERR_ARG;
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (n_fr < 0 || (n_fr > 0 && (!Xfr || ldfr < n_fr || !evals_fr)))
    return fail(c, CHFSI_ERR_ARG, "density: Xfr, ldfr >= n_fr and evals_fr are needed when n_fr > 0");
  if (!rho) return fail(c, CHFSI_ERR_ARG, "density: rho must be a device array of n_dof");
  if (n_fr > 0 && !(sigma > 0)) return fail(c, CHFSI_ERR_ARG, "density: sigma must be positive");
  const int64_t nd = c->mesh.n_dof;
  double *w = nullptr;
  if (n_fr > 0) {
    HIPCHK(c, c->occ_d.ensure((size_t)n_fr * sizeof(double)));
    if (c->host_scratch.size() < (size_t)n_fr) c->host_scratch.resize(n_fr);
    for (int k = 0; k < n_fr; ++k) c->host_scratch[k] = fermi_dirac(evals_fr[k], mu, sigma) - 1.0;
    w = c->occ_d.as<double>();
    HIPCHK(c, hipMemcpyAsync(w, c->host_scratch.data(), n_fr * sizeof(double), hipMemcpyHostToDevice, c->stream));
    // the host staging array is reused by later calls
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  density_launch(X, ld, ncols, Xfr, ldfr, n_fr, w, c->minv64.as<double>(), nd, rho, c->stream);
  HIPCHK(c, hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------
static double elapsed_s(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0;
  return ms * 1e-3;
}

extern "C" int chfsi_solve(chfsi_ctx *c, const chfsi_opts *o, double *X, int64_t ld, double *evals, double *resid,
                           chfsi_report *rep) {
  if (!o) return fail(c, CHFSI_ERR_ARG, "solve: null options");
  const int nb = o->nblock;
  if (int r = check_block(c, X, ld, nb)) return r;
  if (o->nstates < 1 || o->nstates > nb || o->degree < 1 || o->max_iter < 0 || !(o->tol > 0) || !evals || !resid)
    return fail(c, CHFSI_ERR_ARG, "solve: invalid options");
  if (nb > c->mesh.n_dof) return fail(c, CHFSI_ERR_ARG, "solve: more vectors than degrees of freedom");
  if (int r = ensure_small(c, nb)) return r;
  HIPCHK(c, c->HX.ensure((size_t)c->mesh.n_dof * nb * sizeof(double)));
  double *HX = c->HX.as<double>();
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i) HIPCHK(c, hipEventCreate(&ev[i]));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int i = 0; i < 6; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  chfsi_report R;
  std::memset(&R, 0, sizeof R);
  const int nrung = std::max(1, std::min(o->n_ladder, 4));
  auto rung_prec = [&](int rg) { return o->n_ladder > 0 ? o->ladder[rg] : CHFSI_FP64; };
  int rung = 0;
  // mixed CholGS runs on the reduced-precision rungs; with a ladder the last
  // rung is FP64 throughout (FP32 rounding of the overlap inputs leaves a
  // residual floor near 1e-7 relative)
  auto rung_tol = [&](int rg) {
    if (o->ladder_tol[rg] > 0) return o->ladder_tol[rg];
    const chfsi_prec pr = rung_prec(rg);
    const double u = pr == CHFSI_BF16 ? 0x1p-8 : pr == CHFSI_BF16X3 ? 0x1p-16 : pr == CHFSI_FP32 ? 0x1p-24 : 0.0;
    return 4.0 * u * c->ub;
  };
  auto mixed_now = [&]() { return (o->mixed_cholgs && (o->n_ladder <= 1 || rung + 1 < nrung)) ? 1 : 0; };
  int mixed = mixed_now();
  // start: CholGS + RR on the given block
  HIPCHK(c, hipEventRecord(ev[0], c->stream));
  int passes = 0;
  int st = orth_robust(c, X, ld, nb, mixed, &passes);
  if (st) return st;
  HIPCHK(c, hipEventRecord(ev[1], c->stream));
  int rr_st = rr_impl(c, X, ld, nb, HX, nb, evals, resid, nullptr);
  if (rr_st < 0) return rr_st;
  HIPCHK(c, hipEventRecord(ev[2], c->stream));
  HIPCHK(c, hipEventSynchronize(ev[2]));
  R.t_cholgs += elapsed_s(ev[0], ev[1]);
  R.t_rr += elapsed_s(ev[1], ev[2]);
  R.dofvecs += c->mesh.n_dof * (int64_t)nb;
  auto maxres = [&]() {
    double m = 0;
    for (int i = 0; i < o->nstates; ++i) m = std::max(m, resid[i]);
    return m;
  };
  double res = maxres();
  int it = 0;
  while (res > o->tol && it < o->max_iter) {
    const double a = evals[nb - 1], a0 = evals[0], b = c->ub;
    if (!(a0 < a && a < b)) return fail(c, CHFSI_ERR_NONFINITE, "solve: Ritz values outside the filter bounds");
    HIPCHK(c, hipEventRecord(ev[3], c->stream));
    st = chfsi_chebyshev_filter(c, X, ld, nb, o->degree, a, b, a0, rung_prec(rung), o->block_width);
    if (st) return st;
    HIPCHK(c, hipEventRecord(ev[4], c->stream));
    st = orth_robust(c, X, ld, nb, mixed, &passes);
    if (st) return st;
    HIPCHK(c, hipEventRecord(ev[5], c->stream));
    rr_st = rr_impl(c, X, ld, nb, HX, nb, evals, resid, nullptr);
    if (rr_st < 0) return rr_st;
    HIPCHK(c, hipEventRecord(ev[0], c->stream));
    HIPCHK(c, hipEventSynchronize(ev[0]));
    R.t_filter += elapsed_s(ev[3], ev[4]);
    R.t_cholgs += elapsed_s(ev[4], ev[5]);
    R.t_rr += elapsed_s(ev[5], ev[0]);
    R.dofvecs += c->mesh.n_dof * (int64_t)nb * (o->degree + 1);
    ++it;
    const double nres = maxres();
    if (o->n_ladder > 1 && rung + 1 < nrung) {
      const bool stalled = nres > 0.98 * res;
      const bool below = nres < rung_tol(rung);
      if (stalled || below) ++rung;
      mixed = mixed_now();
    }
    res = nres;
    if (c->verbose) {
      std::fprintf(stderr, "[chfsi] pass %d: max wanted residual %.3e, rung %d, filter %.3f s, cholgs %.3f s, rr %.3f s\n",
                   it, res, rung, R.t_filter, R.t_cholgs, R.t_rr);
      std::fflush(stderr);
    }
  }
  R.iters = it;
  R.rung = rung;
  R.max_resid = res;
  // an unconverged projected eigensolve in the last Rayleigh-Ritz leaves
  // approximate Ritz pairs: reported as not converged
  R.status = (res <= o->tol && rr_st == 0) ? CHFSI_OK : CHFSI_WARN_NOT_CONVERGED;
  if (rep) *rep = R;
  return R.status;
}

// ---------------------------------------------------------------------------
// footprint
// ---------------------------------------------------------------------------
extern "C" int chfsi_device_bytes(const chfsi_ctx *c, size_t *bytes) {
  if (!c || !bytes) return CHFSI_ERR_ARG;
  size_t t = 0;
  const_cast<chfsi_ctx *>(c)->each_buf([&t](DevBuf &b) { t += b.bytes; });
  *bytes = t;
  return 0;
}

extern "C" size_t chfsi_footprint_bytes(int n_el, int p, int nblock, int block_width, chfsi_prec prec) {
  if (n_el < 1 || p < 1 || p > 12 || nblock < 1) return 0;
  if (p > 7 && prec != CHFSI_FP64 && prec != CHFSI_FP32) return 0;   // no BF16 kernel above p = 7
  const size_t n = (size_t)n_el * p - 1, nd = n * n * n, ncell = (size_t)n_el * n_el * n_el;
  const size_t nl = (size_t)(p + 1) * (p + 1) * (p + 1), np = (nl + 15) / 16 * 16;
  const size_t npr = p > 7 ? (size_t)hx_rows_padded((int)nl) : np, npb = p > 7 ? 0 : (nl + 31) / 32 * 32;
  const size_t bw = (size_t)std::min(block_width > 0 ? block_width : 128, nblock);
  const size_t elem = prec == CHFSI_FP64 ? 8 : 4;
  size_t b = ncell * nl * 4 + ncell * 4 + np * npr * 12 + nd * 24 + npb * npb * 4;  // tables, K, minv, V
  b += 3 * nd * bw * elem;                                         // filter buffers
  b += nd * nblock * 8;                                            // HX
  const size_t nn = (size_t)nblock * nblock;
  b += 4 * nn * 8 + jacobi_work_elems(nblock) * 8;                 // S, Z, W, jacobi
  b += gram_part_elems_slots((int64_t)nd, nblock, 512) * 8;       // 256 CUs x 2 resident gram work-groups
  b += rmul_scratch_elems((int64_t)nd, nblock) * 8;
  b += (size_t)resid_nchunk((int64_t)nd) * nblock * 8;
  return b;
}
