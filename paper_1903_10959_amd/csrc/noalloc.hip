// CholGS (Alg. 3) for callers that cannot allocate device memory: the same
// kernels as chfsi_orthonormalize, with every workspace carved out of one
// file-scope device array instead of the context's grown-on-demand buffers.
//
// Host code must not pass `scratch` itself to a kernel or a copy: in host code
// the name denotes a host-side stand-in.  Its device address, which differs
// per GPU, is looked up once per device with hipGetSymbolAddress (from
// chfsi_create, with that device current) and kept in g_scratch[device].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "../../include/chfsi.h"
#include "ctx.hpp"
#include "kernels.hpp"

using namespace chfsi;

namespace {

constexpr int MAX_COLS = CHFSI_NOALLOC_MAX_COLS;
constexpr size_t SCRATCH_BYTES = (size_t)CHFSI_NOALLOC_SCRATCH_MIB << 20;
constexpr size_t SCRATCH_ELEMS = SCRATCH_BYTES / sizeof(double);

static __device__ __align__(256) double scratch[SCRATCH_ELEMS];

constexpr int MAX_DEVICES = 64;
std::mutex g_mx;
double *g_scratch[MAX_DEVICES] = {};

// Layout (in doubles, each part 256-byte aligned): S, Z, W (MAX_COLS^2 each),
// the 32x32 diagonal inverses, diag0, minratio, the flag, the rotation panel
// and, for the rest, the overlap's split partials.
constexpr size_t al(size_t e) { return (e + 31) / 32 * 32; }
constexpr size_t NN = (size_t)MAX_COLS * MAX_COLS;
constexpr size_t NB32 = (MAX_COLS + 31) / 32;
constexpr size_t OFF_S = 0, OFF_Z = OFF_S + al(NN), OFF_W = OFF_Z + al(NN), OFF_DINV = OFF_W + al(NN),
                 OFF_DIAG = OFF_DINV + al(NB32 * 32 * 32), OFF_RATIO = OFF_DIAG + al(MAX_COLS),
                 OFF_FLAG = OFF_RATIO + al(NB32), OFF_PANEL = OFF_FLAG + al(4);
constexpr size_t PANEL_ELEMS = (size_t)3 << 20;      // 24 MiB row panel of the rotation
constexpr size_t OFF_PART = OFF_PANEL + al(PANEL_ELEMS);
static_assert(OFF_PART < SCRATCH_ELEMS, "scratch layout");
constexpr size_t PART_ELEMS = SCRATCH_ELEMS - OFF_PART;

}  // namespace

namespace chfsi {
// Device address of this GPU's scratch array, looked up once per device.  The
// caller has made `device` current.
int noalloc_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return CHFSI_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_mx);
  if (g_scratch[device]) return 0;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return CHFSI_ERR_HIP;
  g_scratch[device] = static_cast<double *>(p);
  return 0;
}
}  // namespace chfsi

extern "C" int chfsi_orthonormalize_noalloc(chfsi_ctx *c, double *X, int64_t ld, int ncols, int mixed) {
  if (int r = check_block(c, X, ld, ncols)) return r;
  if (ncols > MAX_COLS) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "orthonormalize_noalloc: %d columns, above the limit of %d", ncols, MAX_COLS);
    return fail(c, CHFSI_ERR_ARG, msg);
  }
  double *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mx);
    base = c->device < MAX_DEVICES ? g_scratch[c->device] : nullptr;
  }
  if (!base) return fail(c, CHFSI_ERR_STATE, "orthonormalize_noalloc: scratch address not set up for this device");
  double host_ratio[NB32];
  CholWs w;
  w.S = base + OFF_S;
  w.Z = base + OFF_Z;
  w.W = base + OFF_W;
  w.dinv = base + OFF_DINV;
  w.diag0 = base + OFF_DIAG;
  w.minratio = base + OFF_RATIO;
  w.flag = reinterpret_cast<int *>(base + OFF_FLAG);
  w.panel = base + OFF_PANEL;
  w.panel_elems = PANEL_ELEMS;
  w.part = base + OFF_PART;
  w.part_elems = PART_ELEMS;
  w.host_ratio = host_ratio;
  return cholgs_core(c, X, ld, ncols, mixed, 0.0, nullptr, w);
}
