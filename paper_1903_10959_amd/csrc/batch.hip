// Batched ChFSI over many independent problems (the paper's k-point groups,
// placed on one device), as a session whose membership changes between passes
// (continuous batching).  One Chebyshev step of every problem in a precision
// group (BF16 / BF16x3, FP32, FP64) runs in shared launches, one per (padded
// cell size, colour), from a device work list of (problem, cell, column tile)
// items.  The degree-m sweep
// of a group is captured once per membership in a HIP graph and replayed each
// pass; only the per-problem recursion coefficients change between passes and
// are copied to the device before the replay.  CholGS and Rayleigh-Ritz run
// per problem on host threads, each problem on its own context and stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <thread>
#include <vector>

#include "ctx.hpp"
#include "kernels.hpp"

using namespace chfsi;

namespace {

struct Prob {
  int id = -1;
  chfsi_ctx *c = nullptr;
  chfsi_opts o;
  double *X = nullptr;
  int64_t ld = 0;
  double *evals = nullptr, *resid = nullptr;
  chfsi_report rep;
  bool started = false, done = false;
  int rung = 0;
  double res = INFINITY;
  bool jac_warn = false;     // the last projected eigensolve ran out of sweeps
};

// Runs fn(i) for every i in [0, n) on up to `threads` host threads, with the
// indices of one group (problems whose contexts share a HIP stream) handled in
// order by one thread, so that no stream is driven by two host threads at
// once.  fn's status for each index goes to st[i].
template <typename F>
void parallel_for_groups(const std::vector<std::vector<int>> &groups, int threads, std::vector<int> &st, F fn) {
  std::atomic<int> next(0);
  const int ng = (int)groups.size();
  auto worker = [&]() {
    for (;;) {
      const int g = next.fetch_add(1);
      if (g >= ng) return;
      for (int i : groups[g]) st[i] = fn(i);
    }
  };
  const int t = std::max(1, std::min(threads, ng));
  std::vector<std::thread> pool;
  for (int k = 1; k < t; ++k) pool.emplace_back(worker);
  worker();
  for (auto &th : pool) th.join();
}

chfsi_prec rung_prec(const Prob &p) { return p.o.n_ladder > 0 ? p.o.ladder[p.rung] : CHFSI_FP64; }
int n_rungs(const Prob &p) { return std::max(1, std::min(p.o.n_ladder, 4)); }
int mixed_now(const Prob &p) {
  return (p.o.mixed_cholgs && (p.o.n_ladder <= 1 || p.rung + 1 < n_rungs(p))) ? 1 : 0;
}
bool bf16_rung(const Prob &p) { return rung_prec(p) == CHFSI_BF16 || rung_prec(p) == CHFSI_BF16X3; }
double rung_tol(const Prob &p) {
  if (p.o.ladder_tol[p.rung] > 0) return p.o.ladder_tol[p.rung];
  const chfsi_prec pr = rung_prec(p);
  const double u = pr == CHFSI_BF16 ? 0x1p-8 : pr == CHFSI_BF16X3 ? 0x1p-16 : pr == CHFSI_FP32 ? 0x1p-24 : 0.0;
  return 4.0 * u * p.c->ub;
}
double max_wanted(const Prob &p) {
  double m = 0;
  for (int i = 0; i < p.o.nstates; ++i) m = std::max(m, p.resid[i]);
  return m;
}

// recursion roles at step k: (cur, prev, out) of the three buffers
void roles(int degree, std::vector<int> &cur, std::vector<int> &prev, std::vector<int> &out, int &final_buf) {
  int c = 0, p = -1;
  cur.clear();
  prev.clear();
  out.clear();
  for (int k = 0; k < degree; ++k) {
    int o = 0;
    while (o == c || o == p) ++o;
    cur.push_back(c);
    prev.push_back(p);
    out.push_back(o);
    p = c;
    c = o;
  }
  final_buf = c;
}

template <typename T>
struct Sweep {
  DevBuf probs, work, coef;
  std::vector<int> members;      // problem ids of the captured graph (BF16: 2 id + split)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<T> hcoef;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    members.clear();
  }
  void release() {
    drop_graph();
    probs.release();
    work.release();
    coef.release();
  }
};

}  // namespace

struct chfsi_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int degree = 0;
  std::vector<Prob> probs;       // indexed by id
  std::deque<int> finished;      // ids that left and are not reported yet
  Sweep<double> s64;
  Sweep<float> s32;
  Sweep<float> sbf;              // BF16 and BF16x3 rungs (FP32 recursion state)
  bool verbose = false;
  int threads = 8;               // host threads for the per-problem CholGS / Rayleigh-Ritz
  // shared Jacobi eigensolve of the projected Hamiltonians
  chfsi::DevBuf jac_table, jac_norms;
  std::vector<double> jac_host;
  double build_ms = 0;           // host time spent (re)building sweep graphs in the current pass
};

namespace {

int bfail(chfsi_batch *b, int code, const std::string &msg) {
  if (b) b->err = msg;
  return code;
}

// A problem leaves the session: converged, out of passes, or failed (status < 0).
void finish_prob(chfsi_batch *B, Prob &p, int fail_status = 0) {
  p.done = true;
  p.rep.max_resid = p.res;
  p.rep.rung = p.rung;
  if (fail_status < 0) p.rep.status = fail_status;
  else p.rep.status = (p.res <= p.o.tol && !p.jac_warn) ? CHFSI_OK : CHFSI_WARN_NOT_CONVERGED;
  B->finished.push_back(p.id);
}

// Problems of ids grouped by the HIP stream of their context (positions into ids).
std::vector<std::vector<int>> stream_groups(chfsi_batch *B, const std::vector<int> &ids) {
  std::vector<std::vector<int>> groups;
  std::map<hipStream_t, int> where;
  for (int i = 0; i < (int)ids.size(); ++i) {
    hipStream_t s = B->probs[ids[i]].c->stream;
    auto it = where.find(s);
    if (it == where.end()) {
      where[s] = (int)groups.size();
      groups.push_back({i});
    } else {
      groups[it->second].push_back(i);
    }
  }
  return groups;
}

#define BCHK(b, call)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return bfail(b, e_ == hipErrorOutOfMemory ? CHFSI_ERR_OOM : CHFSI_ERR_HIP,                   \
                   std::string(#call) + ": " + hipGetErrorString(e_));                             \
  } while (0)

template <typename T>
int build_sweep(chfsi_batch *B, Sweep<T> &S, const std::vector<int> &ids, const std::vector<int> &key) {
  S.drop_graph();
  if (ids.empty()) return 0;
  const bool f64 = sizeof(T) == 8;
  std::vector<BatchProblem<T>> hp;
  // (np, (tile variant + 1) * 8 + cells per tile, colour) -> work items
  std::map<std::tuple<int, int, int>, std::vector<int4>> lists;
  for (size_t m = 0; m < ids.size(); ++m) {
    Prob &p = B->probs[ids[m]];
    chfsi_ctx *c = p.c;
    const int nb = p.o.nblock;
    BatchProblem<T> P;
    P.buf[0] = f64 ? (T *)p.X : c->fbuf[0].as<T>();
    P.ld[0] = f64 ? p.ld : nb;
    P.buf[1] = c->fbuf[1].as<T>();
    P.buf[2] = c->fbuf[2].as<T>();
    P.ld[1] = P.ld[2] = nb;
    P.K = f64 ? (const T *)c->K64.p : (const T *)c->K32.p;
    P.cmap = c->cmap.as<int32_t>();
    P.minv = f64 ? (const T *)c->minv64.p : (const T *)c->minv32.p;
    P.V = f64 ? (const T *)c->V64.p : (const T *)c->V32.p;
    P.coef = nullptr;
    P.cells = c->cells.as<int32_t>();
    P.n_loc = c->mesh.n_loc;
    P.q = c->mesh.q;
    P.n_el = c->mesh.n_el;
    P.ncols = nb;
    hp.push_back(P);
    const int cpt = cells_per_tile(c, nb, hx_tile_width<T>(c->mesh.np, c->tile_variant, 1));
    const int cw = hx_tile_width<T>(c->mesh.np, c->tile_variant, cpt);
    if (cw <= 0) return bfail(B, CHFSI_ERR_ARG, "batch: no cell kernel for a problem's degree");
    const int ntiles = (nb + cw - 1) / cw;
    for (int col = 0; col < 8; ++col) {
      const int e0 = c->mesh.color_offset[col], e1 = c->mesh.color_offset[col + 1];
      for (int s = e0; s < e1; s += cpt)
        for (int t = 0; t < ntiles; ++t)
          lists[{c->mesh.np, (c->tile_variant + 1) * 8 + cpt, col}].push_back(
              make_int4((int)m, s, t, std::min(cpt, e1 - s)));
    }
  }
  BCHK(B, S.coef.ensure((size_t)3 * B->degree * ids.size() * sizeof(T)));
  for (size_t m = 0; m < hp.size(); ++m) hp[m].coef = S.coef.template as<T>() + (size_t)3 * B->degree * m;
  std::vector<int4> all;
  std::vector<std::tuple<int, int, int>> groups;  // (np, (tile variant + 1) * 8 + cells per tile, offset)
  std::vector<int> counts;
  // colour-major launch order: every problem sees its colours in order 0..7
  for (int col = 0; col < 8; ++col)
    for (auto &kv : lists)
      if (std::get<2>(kv.first) == col) {
        groups.push_back({std::get<0>(kv.first), std::get<1>(kv.first), (int)all.size()});
        counts.push_back((int)kv.second.size());
        all.insert(all.end(), kv.second.begin(), kv.second.end());
      }
  BCHK(B, S.probs.ensure(hp.size() * sizeof(BatchProblem<T>)));
  BCHK(B, S.work.ensure(all.size() * sizeof(int4)));
  BCHK(B, hipMemcpyAsync(S.probs.p, hp.data(), hp.size() * sizeof(BatchProblem<T>), hipMemcpyHostToDevice, B->stream));
  BCHK(B, hipMemcpyAsync(S.work.p, all.data(), all.size() * sizeof(int4), hipMemcpyHostToDevice, B->stream));
  BCHK(B, hipStreamSynchronize(B->stream));
  std::vector<int> cur, prev, out;
  int final_buf = 0;
  roles(B->degree, cur, prev, out, final_buf);
  BCHK(B, hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
  if (!f64)
    for (int id : ids) {
      Prob &p = B->probs[id];
      copy_cols_launch<double, float>(p.X, p.ld, p.c->fbuf[0].as<float>(), p.o.nblock, p.c->mesh.n_dof, p.o.nblock,
                                      B->stream);
    }
  int lerr = 0;
  for (int k = 0; k < B->degree; ++k)
    for (size_t g = 0; g < groups.size(); ++g)
      lerr |= hx_cells_batch_launch<T>(std::get<0>(groups[g]), std::get<1>(groups[g]) / 8 - 1,
                                       std::get<1>(groups[g]) % 8, S.probs.template as<BatchProblem<T>>(),
                                       S.work.template as<int4>() + std::get<2>(groups[g]), counts[g], k, cur[k],
                                       prev[k], out[k], B->stream);
  for (size_t m = 0; m < ids.size(); ++m) {
    Prob &p = B->probs[ids[m]];
    if (!f64)
      copy_cols_launch<float, double>((const float *)hp[m].buf[final_buf], hp[m].ld[final_buf], p.X, p.ld,
                                      p.c->mesh.n_dof, p.o.nblock, B->stream);
    else if (final_buf != 0)
      copy_cols_launch<double, double>((const double *)hp[m].buf[final_buf], hp[m].ld[final_buf], p.X, p.ld,
                                       p.c->mesh.n_dof, p.o.nblock, B->stream);
  }
  hipError_t ce = hipStreamEndCapture(B->stream, &S.graph);
  if (ce != hipSuccess) return bfail(B, CHFSI_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  if (lerr) return bfail(B, CHFSI_ERR_ARG, "batch: no cell kernel for a problem's degree");
  BCHK(B, hipGraphInstantiate(&S.exec, S.graph, nullptr, nullptr, 0));
  S.members = key;
  return 0;
}

// The BF16 sweep: BF16 (or hi/lo split) cell products on FP32 recursion
// state, one launch per (padded size, split, colour) and step; one cell x 64
// columns per work item.
int build_sweep_bf16(chfsi_batch *B, Sweep<float> &S, const std::vector<int> &ids, const std::vector<int> &key) {
  S.drop_graph();
  if (ids.empty()) return 0;
  constexpr int TWB = 64;
  std::vector<BatchProblemBf16> hp;
  // (npb, split, colour) -> work items
  std::map<std::tuple<int, int, int>, std::vector<int4>> lists;
  for (size_t m = 0; m < ids.size(); ++m) {
    Prob &p = B->probs[ids[m]];
    chfsi_ctx *c = p.c;
    const int nb = p.o.nblock;
    if (c->npb <= 0) return bfail(B, CHFSI_ERR_ARG, "batch: no BF16 cell kernel for a problem's degree");
    BatchProblemBf16 P;
    for (int k = 0; k < 3; ++k) {
      P.buf[k] = c->fbuf[k].as<float>();
      P.ld[k] = nb;
    }
    P.Kh = c->Kbh.as<const __bf16>();
    P.Kl = c->Kbl.as<const __bf16>();
    P.cmap = c->cmap.as<int32_t>();
    P.cells = c->cells.as<int32_t>();
    P.minv = c->minv32.as<float>();
    P.V = c->V32.as<float>();
    P.coef = nullptr;
    P.n_loc = c->mesh.n_loc;
    P.q = c->mesh.q;
    P.n_el = c->mesh.n_el;
    P.ncols = nb;
    hp.push_back(P);
    const int split = rung_prec(p) == CHFSI_BF16X3 ? 1 : 0;
    const int ntiles = (nb + TWB - 1) / TWB;
    for (int col = 0; col < 8; ++col)
      for (int e = c->mesh.color_offset[col]; e < c->mesh.color_offset[col + 1]; ++e)
        for (int t = 0; t < ntiles; ++t) lists[{c->npb, split, col}].push_back(make_int4((int)m, e, t, 1));
  }
  BCHK(B, S.coef.ensure((size_t)3 * B->degree * ids.size() * sizeof(float)));
  for (size_t m = 0; m < hp.size(); ++m) hp[m].coef = S.coef.as<float>() + (size_t)3 * B->degree * m;
  std::vector<int4> all;
  std::vector<std::tuple<int, int, int>> groups;  // (npb, split, offset)
  std::vector<int> counts;
  for (int col = 0; col < 8; ++col)
    for (auto &kv : lists)
      if (std::get<2>(kv.first) == col) {
        groups.push_back({std::get<0>(kv.first), std::get<1>(kv.first), (int)all.size()});
        counts.push_back((int)kv.second.size());
        all.insert(all.end(), kv.second.begin(), kv.second.end());
      }
  BCHK(B, S.probs.ensure(hp.size() * sizeof(BatchProblemBf16)));
  BCHK(B, S.work.ensure(all.size() * sizeof(int4)));
  BCHK(B, hipMemcpyAsync(S.probs.p, hp.data(), hp.size() * sizeof(BatchProblemBf16), hipMemcpyHostToDevice,
                         B->stream));
  BCHK(B, hipMemcpyAsync(S.work.p, all.data(), all.size() * sizeof(int4), hipMemcpyHostToDevice, B->stream));
  BCHK(B, hipStreamSynchronize(B->stream));
  std::vector<int> cur, prev, out;
  int final_buf = 0;
  roles(B->degree, cur, prev, out, final_buf);
  BCHK(B, hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
  for (int id : ids) {
    Prob &p = B->probs[id];
    copy_cols_launch<double, float>(p.X, p.ld, p.c->fbuf[0].as<float>(), p.o.nblock, p.c->mesh.n_dof, p.o.nblock,
                                    B->stream);
  }
  int lerr = 0;
  for (int k = 0; k < B->degree; ++k)
    for (size_t g = 0; g < groups.size(); ++g)
      lerr |= hx_cells_bf16_batch_launch(std::get<0>(groups[g]), std::get<1>(groups[g]),
                                         S.probs.as<BatchProblemBf16>(), S.work.as<int4>() + std::get<2>(groups[g]),
                                         counts[g], k, cur[k], prev[k], out[k], B->stream);
  for (size_t m = 0; m < ids.size(); ++m) {
    Prob &p = B->probs[ids[m]];
    copy_cols_launch<float, double>((const float *)hp[m].buf[final_buf], hp[m].ld[final_buf], p.X, p.ld,
                                    p.c->mesh.n_dof, p.o.nblock, B->stream);
  }
  hipError_t ce = hipStreamEndCapture(B->stream, &S.graph);
  if (ce != hipSuccess) return bfail(B, CHFSI_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  if (lerr) return bfail(B, CHFSI_ERR_ARG, "batch: no BF16 cell kernel for a problem's degree");
  BCHK(B, hipGraphInstantiate(&S.exec, S.graph, nullptr, nullptr, 0));
  S.members = key;
  return 0;
}

// One pass of a precision group's sweep: (re)captures the graph when the
// membership (for the BF16 group: with each member's split) changed, then
// uploads the recursion coefficients and replays it.
template <typename T>
int run_sweep(chfsi_batch *B, Sweep<T> &S, const std::vector<int> &ids, float *ms_out, bool bf16 = false) {
  *ms_out = 0;
  if (ids.empty()) return 0;
  std::vector<int> key(ids);
  if (bf16)
    for (size_t m = 0; m < ids.size(); ++m) key[m] = 2 * ids[m] + (rung_prec(B->probs[ids[m]]) == CHFSI_BF16X3);
  if (key != S.members) {
    const auto t0 = std::chrono::steady_clock::now();
    int r;
    if constexpr (sizeof(T) == 4) r = bf16 ? build_sweep_bf16(B, S, ids, key) : build_sweep<T>(B, S, ids, key);
    else r = build_sweep<T>(B, S, ids, key);
    if (r) return r;
    B->build_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  const int m_deg = B->degree;
  S.hcoef.assign((size_t)3 * m_deg * ids.size(), T(0));
  for (size_t m = 0; m < ids.size(); ++m) {
    Prob &p = B->probs[ids[m]];
    const int nb = p.o.nblock;
    const double a = p.evals[nb - 1], a0 = p.evals[0], b = p.c->ub;
    if (!(a0 < a && a < b)) return bfail(B, CHFSI_ERR_STATE, "batch: internal: unchecked filter bounds");
    // normalised recursion: rho_1 = 1/xi0, rho_{k+1} = 1/(2 xi0 - rho_k)
    const double cc = 0.5 * (a + b), e = 0.5 * (b - a), xi0 = (a0 - cc) / e;
    double rho = 1.0 / xi0;
    T *tc = S.hcoef.data() + (size_t)3 * m_deg * m;
    for (int k = 0; k < m_deg; ++k) {
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
      tc[3 * k] = (T)s1;
      tc[3 * k + 1] = (T)s2;
      tc[3 * k + 2] = (T)cc;
    }
  }
  BCHK(B, hipMemcpyAsync(S.coef.p, S.hcoef.data(), S.hcoef.size() * sizeof(T), hipMemcpyHostToDevice, B->stream));
  hipEvent_t e0, e1;
  BCHK(B, hipEventCreate(&e0));
  BCHK(B, hipEventCreate(&e1));
  (void)hipEventRecord(e0, B->stream);
  hipError_t le = hipGraphLaunch(S.exec, B->stream);
  (void)hipEventRecord(e1, B->stream);
  hipError_t se = hipStreamSynchronize(B->stream);
  (void)hipEventElapsedTime(ms_out, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (le != hipSuccess || se != hipSuccess)
    return bfail(B, CHFSI_ERR_HIP, std::string("batch sweep: ") + hipGetErrorString(le != hipSuccess ? le : se));
  return 0;
}

// CholGS + Rayleigh-Ritz of many problems: CholGS and the projection per
// problem on its own stream (host threads), one batched Jacobi eigensolve of
// all projected Hamiltonians on the batch stream, then the rotations and
// residuals per problem.  A problem whose own step fails (a non-positive-
// definite overlap, a HIP error on its stream) leaves the session with that
// status; the others go on.  Returns non-zero only for a failure of the
// shared eigensolve.
int subspace_steps(chfsi_batch *B, const std::vector<int> &ids_in, bool filtered) {
  std::vector<int> ids(ids_in);
  if (ids.empty()) return 0;
  std::vector<int> st(ids.size(), 0);
  parallel_for_groups(stream_groups(B, ids), B->threads, st, [&](int i) {
    Prob &p = B->probs[ids[i]];
    if (int r = set_dev(p.c)) return r;
    int passes = 0;
    if (int r = orth_robust(p.c, p.X, p.ld, p.o.nblock, filtered ? mixed_now(p) : 0, &passes)) return r;
    if (int r = rr_project(p.c, p.X, p.ld, p.o.nblock, p.c->HX.as<double>(), p.o.nblock)) return r;
    return hipStreamSynchronize(p.c->stream) == hipSuccess ? 0 : (int)CHFSI_ERR_HIP;
  });
  std::vector<int> keep;
  for (size_t i = 0; i < ids.size(); ++i) {
    if (st[i] != 0) finish_prob(B, B->probs[ids[i]], st[i] < 0 ? st[i] : CHFSI_ERR_HIP);
    else keep.push_back(ids[i]);
  }
  ids.swap(keep);
  if (ids.empty()) return 0;
  std::vector<JacobiJob> jobs;
  for (int id : ids) jobs.push_back(rr_eigen_job(B->probs[id].c, B->probs[id].o.nblock));
  BCHK(B, B->jac_table.ensure(jacobi_table_bytes((int)jobs.size())));
  BCHK(B, B->jac_norms.ensure(jacobi_norms_elems((int)jobs.size()) * sizeof(double)));
  B->jac_host.resize(jacobi_norms_elems((int)jobs.size()));
  std::vector<int> jconv(jobs.size(), 1);
  const int jmax = B->probs[ids[0]].c->jac_sweeps;
  if (jacobi_eigh_batch(jobs.data(), (int)jobs.size(), 1e-14, jmax, B->jac_table.p, B->jac_norms.as<double>(),
                        B->jac_host.data(), B->stream, nullptr, jconv.data()) < 0)
    return bfail(B, CHFSI_ERR_HIP, "batch: Jacobi eigensolve failed");
  BCHK(B, hipStreamSynchronize(B->stream));
  st.assign(ids.size(), 0);
  parallel_for_groups(stream_groups(B, ids), B->threads, st, [&](int i) {
    Prob &p = B->probs[ids[i]];
    if (int r = set_dev(p.c)) return r;
    if (int r = rr_finish(p.c, p.X, p.ld, p.o.nblock, p.c->HX.as<double>(), p.o.nblock, p.evals, p.resid))
      return r;
    p.jac_warn = jconv[i] == 0;
    const double nres = max_wanted(p);
    if (filtered) {
      p.rep.iters++;
      p.rep.dofvecs += p.c->mesh.n_dof * (int64_t)p.o.nblock;
      if (p.rung + 1 < n_rungs(p) && (nres > 0.98 * p.res || nres < rung_tol(p))) ++p.rung;
    } else {
      p.rep.dofvecs += p.c->mesh.n_dof * (int64_t)p.o.nblock;
    }
    p.res = nres;
    return 0;
  });
  for (size_t i = 0; i < ids.size(); ++i)
    if (st[i] != 0) finish_prob(B, B->probs[ids[i]], st[i] < 0 ? st[i] : CHFSI_ERR_HIP);
  return 0;
}

}  // namespace

extern "C" int chfsi_batch_create(chfsi_batch **out, int device) {
  if (!out) return CHFSI_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CHFSI_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return CHFSI_ERR_HIP;
  chfsi_batch *b = new (std::nothrow) chfsi_batch();
  if (!b) return CHFSI_ERR_OOM;
  b->device = device;
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return CHFSI_ERR_HIP;
  }
  const char *v = std::getenv("CHFSI_VERBOSE");
  b->verbose = v && v[0] && v[0] != '0';
  if (const char *t = std::getenv("CHFSI_BATCH_THREADS")) {
    const int n = std::atoi(t);
    if (n >= 1 && n <= 256) b->threads = n;
  }
  *out = b;
  return 0;
}

extern "C" int chfsi_batch_destroy(chfsi_batch *b) {
  if (!b) return CHFSI_ERR_ARG;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  b->s64.release();
  b->s32.release();
  b->sbf.release();
  b->jac_table.release();
  b->jac_norms.release();
  (void)hipStreamDestroy(b->stream);
  delete b;
  return 0;
}

extern "C" const char *chfsi_batch_last_error(const chfsi_batch *b) { return b ? b->err.c_str() : "null batch"; }

extern "C" int chfsi_batch_add(chfsi_batch *b, chfsi_ctx *c, const chfsi_opts *o, double *X, int64_t ld,
                               double *evals, double *resid) {
  if (!b || !c || !o) return CHFSI_ERR_ARG;
  if (c->device != b->device) return bfail(b, CHFSI_ERR_ARG, "batch: context on another device");
  if (int r = check_block(c, X, ld, o->nblock)) return bfail(b, r, "batch: " + c->err);
  if (o->nstates < 1 || o->nstates > o->nblock || o->degree < 1 || o->max_iter < 0 || !(o->tol > 0) || !evals ||
      !resid || o->nblock > c->mesh.n_dof)
    return bfail(b, CHFSI_ERR_ARG, "batch: invalid options");
  if (b->degree == 0) b->degree = o->degree;
  if (o->degree != b->degree) return bfail(b, CHFSI_ERR_ARG, "batch: every problem needs the session's degree");
  for (int k = 0; k < std::max(1, std::min(o->n_ladder, 4)); ++k) {
    const chfsi_prec pr = o->n_ladder > 0 ? o->ladder[k] : CHFSI_FP64;
    if (pr != CHFSI_FP64 && pr != CHFSI_FP32 && pr != CHFSI_BF16 && pr != CHFSI_BF16X3)
      return bfail(b, CHFSI_ERR_ARG, "batch: unknown ladder precision");
    if ((pr == CHFSI_BF16 || pr == CHFSI_BF16X3) && c->npb <= 0)
      return bfail(b, CHFSI_ERR_ARG, "batch: BF16 rungs need degree p <= 7");
  }
  for (const Prob &p : b->probs)
    if (!p.done && p.c == c) return bfail(b, CHFSI_ERR_ARG, "batch: the context is already in the session");
  if (int r = ensure_small(c, o->nblock)) return bfail(b, r, "batch: " + c->err);
  const size_t bytes = (size_t)c->mesh.n_dof * o->nblock * sizeof(double);  // FP64-sized for any rung
  for (int k = 0; k < 3; ++k)
    if (c->fbuf[k].ensure(bytes) != hipSuccess) return bfail(b, CHFSI_ERR_OOM, "batch: filter buffers");
  if (c->HX.ensure(bytes) != hipSuccess) return bfail(b, CHFSI_ERR_OOM, "batch: HX buffer");
  Prob p;
  p.id = (int)b->probs.size();
  p.c = c;
  p.o = *o;
  p.X = X;
  p.ld = ld;
  p.evals = evals;
  p.resid = resid;
  std::memset(&p.rep, 0, sizeof p.rep);
  b->probs.push_back(p);
  return p.id;
}

extern "C" int chfsi_batch_report(const chfsi_batch *b, int id, chfsi_report *rep) {
  if (!b || !rep || id < 0 || id >= (int)b->probs.size()) return CHFSI_ERR_ARG;
  *rep = b->probs[id].rep;
  return 0;
}

extern "C" int chfsi_batch_pass(chfsi_batch *b, int *done_ids, int *n_done, int max_done) {
  if (!b || !n_done || max_done < 0 || (max_done > 0 && !done_ids)) return CHFSI_ERR_ARG;
  if (hipSetDevice(b->device) != hipSuccess) return bfail(b, CHFSI_ERR_HIP, "hipSetDevice");
  // 1. new problems: CholGS + RR of their start block
  std::vector<int> fresh;
  for (Prob &p : b->probs)
    if (!p.done && !p.started) fresh.push_back(p.id);
  if (int st = subspace_steps(b, fresh, false)) return st;
  for (int id : fresh) {
    Prob &p = b->probs[id];
    p.started = true;
    if (!p.done && (p.res <= p.o.tol || p.o.max_iter == 0)) finish_prob(b, p);
  }
  // 2. filter sweeps, one per precision group; a problem whose Ritz values do
  // not give valid filter bounds (a0 < a < b) leaves with CHFSI_ERR_NONFINITE
  std::vector<int> gbf, g32, g64;
  for (Prob &p : b->probs) {
    if (p.done) continue;
    const int nb = p.o.nblock;
    const double a = p.evals[nb - 1], a0 = p.evals[0], ub = p.c->ub;
    if (!(a0 < a && a < ub)) {
      finish_prob(b, p, CHFSI_ERR_NONFINITE);
      continue;
    }
    (bf16_rung(p) ? gbf : rung_prec(p) == CHFSI_FP32 ? g32 : g64).push_back(p.id);
  }
  float msbf = 0, ms32 = 0, ms64 = 0;
  b->build_ms = 0;
  const auto t_sw = std::chrono::steady_clock::now();
  if (int r = run_sweep<float>(b, b->sbf, gbf, &msbf, true)) return r;
  if (int r = run_sweep<float>(b, b->s32, g32, &ms32)) return r;
  if (int r = run_sweep<double>(b, b->s64, g64, &ms64)) return r;
  // 3. CholGS + RR of every swept problem
  std::vector<int> swept(gbf);
  swept.insert(swept.end(), g32.begin(), g32.end());
  swept.insert(swept.end(), g64.begin(), g64.end());
  for (int id : swept) {
    Prob &p = b->probs[id];
    p.rep.t_filter += (bf16_rung(p) ? msbf : rung_prec(p) == CHFSI_FP32 ? ms32 : ms64) * 1e-3;
    p.rep.dofvecs += p.c->mesh.n_dof * (int64_t)p.o.nblock * b->degree;
  }
  const auto t_ss = std::chrono::steady_clock::now();
  if (int st = subspace_steps(b, swept, true)) return st;
  const auto t_end = std::chrono::steady_clock::now();
  int remaining = 0;
  for (int id : swept) {
    Prob &p = b->probs[id];
    if (p.done) continue;                         // failed in its CholGS / Rayleigh-Ritz
    if (p.res <= p.o.tol || p.rep.iters >= p.o.max_iter) finish_prob(b, p);
    else ++remaining;
  }
  if (b->verbose) {
    double worst = 0;
    for (int id : swept) worst = std::max(worst, b->probs[id].res);
    std::fprintf(stderr,
                 "[chfsi] batch pass: %zu BF16 + %zu FP32 + %zu FP64 problems swept (%.2f + %.2f + %.2f ms on the "
                 "device, %.2f ms wall incl. %.2f ms graph builds), CholGS/RR %.2f ms, %d remain, max residual %.3e\n",
                 gbf.size(), g32.size(), g64.size(), msbf, ms32, ms64,
                 std::chrono::duration<double, std::milli>(t_ss - t_sw).count(), b->build_ms,
                 std::chrono::duration<double, std::milli>(t_end - t_ss).count(), remaining, worst);
    std::fflush(stderr);
  }
  int nd = 0;
  while (nd < max_done && !b->finished.empty()) {
    done_ids[nd++] = b->finished.front();
    b->finished.pop_front();
  }
  *n_done = nd;
  return remaining;
}

extern "C" int chfsi_solve_batch(chfsi_ctx *const *ctxs, int n, const chfsi_opts *opts, double *const *X,
                                 const int64_t *ld, double *const *evals, double *const *resid, chfsi_report *reps) {
  if (!ctxs || n < 1 || !opts || !X || !ld || !evals || !resid || !ctxs[0]) return CHFSI_ERR_ARG;
  chfsi_ctx *c0 = ctxs[0];
  chfsi_batch *b = nullptr;
  int st = chfsi_batch_create(&b, c0->device);
  if (st) return fail(c0, st, "batch: cannot create a session");
  struct Guard {
    chfsi_batch *b;
    ~Guard() { chfsi_batch_destroy(b); }
  } g{b};
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return fail(c0, CHFSI_ERR_ARG, "batch: null context");
    const int id = chfsi_batch_add(b, ctxs[i], &opts[i], X[i], ld[i], evals[i], resid[i]);
    if (id < 0) return fail(c0, id, b->err);
  }
  std::vector<int> done(n);
  int nd = 0;
  for (;;) {
    const int rem = chfsi_batch_pass(b, done.data(), &nd, n);
    if (rem < 0) return fail(c0, rem, b->err);
    if (rem == 0) break;
  }
  int worst = CHFSI_OK;
  for (int i = 0; i < n; ++i) {
    const chfsi_report &r = b->probs[i].rep;
    if (r.status != CHFSI_OK) worst = CHFSI_WARN_NOT_CONVERGED;
    if (reps) reps[i] = r;
  }
  return worst;
}

extern "C" int chfsi_batch_set_threads(chfsi_batch *b, int threads) {
  if (!b) return CHFSI_ERR_ARG;
  if (threads < 1 || threads > 256) return bfail(b, CHFSI_ERR_ARG, "batch: threads must be in 1..256");
  b->threads = threads;
  return 0;
}

extern "C" size_t chfsi_batch_footprint_bytes(int n_el, int p, int nblock) {
  if (n_el < 1 || p < 1 || p > 7 || nblock < 1) return 0;
  const size_t n = (size_t)n_el * p - 1, nd = n * n * n, ncell = (size_t)n_el * n_el * n_el;
  if (nd < (size_t)nblock) return 0;
  const size_t nl = (size_t)(p + 1) * (p + 1) * (p + 1), np = (nl + 15) / 16 * 16, npb = (nl + 31) / 32 * 32;
  const size_t nb = (size_t)nblock, nb32 = (nb + 31) / 32;
  // mesh and potential tables (set_mesh, set_potential)
  size_t b = ncell * nl * 4 + ncell * 4 + np * np * 12 + nd * 24 + npb * npb * 4;
  // workspaces of the CholGS / Rayleigh-Ritz steps (ensure_small)
  b += 3 * nb * nb * 8 + nb32 * 32 * 32 * 8 + jacobi_work_elems(nblock) * 8 + 3 * nb * 8 + 4 * sizeof(int) +
       nb32 * 8;
  b += rmul_scratch_elems((int64_t)nd, nblock) * 8;
  b += gram_part_elems_slots((int64_t)nd, nblock, 512) * 8;       // 256 CUs x 2 resident gram work-groups
  b += (size_t)resid_nchunk((int64_t)nd) * nb * 8;
  // the session's three recursion buffers (FP64-sized for either rung) and HX
  b += 4 * nd * nb * 8;
  return b;
}
