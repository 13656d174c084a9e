// Batched ChFSI over many independent problems (the paper's k-point groups on
// one device): one Chebyshev step of every active problem runs in shared
// launches, one per (padded cell size, colour), from a device work list of
// (problem, cell, column tile) items.  The whole degree-m sweep of an active
// set is captured once in a HIP graph and replayed every pass; only the
// per-problem recursion coefficients change between passes and are copied to
// the device before each replay.  CholGS and Rayleigh-Ritz run per problem on
// host threads, each problem on its own context (and stream).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <thread>
#include <vector>

#include "ctx.hpp"
#include "kernels.hpp"

using namespace chfsi;

namespace {

struct Item {
  int idx;          // problem index in the batch
  chfsi_ctx *c;
  const chfsi_opts *o;
  double *X;
  int64_t ld;
  double *evals, *resid;
  chfsi_report rep;
  int status = 0;
  bool active = true;
  double res = INFINITY;
};

// run fn(i) for i in [0, n) on up to `threads` host threads; returns the
// first non-zero status
template <typename F>
int parallel_for(int n, int threads, F fn) {
  std::atomic<int> next(0), first_err(0);
  auto worker = [&]() {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n) return;
      const int st = fn(i);
      if (st != 0) {
        int z = 0;
        first_err.compare_exchange_strong(z, st);
      }
    }
  };
  const int t = std::max(1, std::min(threads, n));
  std::vector<std::thread> pool;
  for (int k = 1; k < t; ++k) pool.emplace_back(worker);
  worker();
  for (auto &th : pool) th.join();
  return first_err.load();
}

double max_wanted(const Item &it) {
  double m = 0;
  for (int i = 0; i < it.o->nstates; ++i) m = std::max(m, it.resid[i]);
  return m;
}

template <typename T>
struct Sweep {
  int degree = 0;
  hipStream_t stream = nullptr;
  DevBuf probs, work, coef;
  std::vector<int> members;                          // item indices in this active set
  std::vector<std::pair<int, int>> groups;           // (np, colour) -> launch
  std::vector<int> goff, gcnt;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int final_buf = 0;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~Sweep() {
    drop_graph();
    probs.release();
    work.release();
    coef.release();
  }
};

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
int build_sweep(Sweep<T> &S, std::vector<Item> &items, chfsi_ctx *c0) {
  S.drop_graph();
  S.members.clear();
  for (auto &it : items)
    if (it.active) S.members.push_back(it.idx);
  if (S.members.empty()) return 0;
  // descriptors
  std::vector<BatchProblem<T>> hp;
  std::map<std::pair<int, int>, std::vector<int4>> lists;  // (np, colour) -> items
  size_t coef_elems = 0;
  for (size_t m = 0; m < S.members.size(); ++m) {
    Item &it = items[S.members[m]];
    chfsi_ctx *c = it.c;
    const int nb = it.o->nblock;
    BatchProblem<T> P;
    const bool f64 = sizeof(T) == 8;
    P.buf[0] = f64 ? (T *)it.X : c->fbuf[0].as<T>();
    P.ld[0] = f64 ? it.ld : nb;
    P.buf[1] = c->fbuf[1].as<T>();
    P.buf[2] = c->fbuf[2].as<T>();
    P.ld[1] = P.ld[2] = nb;
    P.K = f64 ? (const T *)c->K64.p : (const T *)c->K32.p;
    P.cmap = c->cmap.as<int32_t>();
    P.minv = f64 ? (const T *)c->minv64.p : (const T *)c->minv32.p;
    P.V = f64 ? (const T *)c->V64.p : (const T *)c->V32.p;
    P.coef = nullptr;  // set after the coefficient buffer exists
    P.n_loc = c->mesh.n_loc;
    P.q = c->mesh.q;
    P.n_el = c->mesh.n_el;
    P.ncols = nb;
    hp.push_back(P);
    coef_elems += (size_t)3 * S.degree;
    const int ntiles = (nb + 63) / 64;
    for (int col = 0; col < 8; ++col)
      for (int s = c->mesh.color_offset[col]; s < c->mesh.color_offset[col + 1]; ++s)
        for (int t = 0; t < ntiles; ++t)
          lists[{c->mesh.np, col}].push_back(make_int4((int)m, c->mesh.cell_order[s], t, 0));
  }
  HIPCHK(c0, S.coef.ensure(coef_elems * sizeof(T)));
  for (size_t m = 0; m < hp.size(); ++m) hp[m].coef = S.coef.template as<T>() + (size_t)3 * S.degree * m;
  std::vector<int4> all;
  S.groups.clear();
  S.goff.clear();
  S.gcnt.clear();
  // launch order: colour-major, so every problem sees its colours in order
  for (int col = 0; col < 8; ++col)
    for (auto &kv : lists)
      if (kv.first.second == col) {
        S.groups.push_back(kv.first);
        S.goff.push_back((int)all.size());
        S.gcnt.push_back((int)kv.second.size());
        all.insert(all.end(), kv.second.begin(), kv.second.end());
      }
  HIPCHK(c0, S.probs.ensure(hp.size() * sizeof(BatchProblem<T>)));
  HIPCHK(c0, S.work.ensure(all.size() * sizeof(int4)));
  HIPCHK(c0, hipMemcpyAsync(S.probs.p, hp.data(), hp.size() * sizeof(BatchProblem<T>), hipMemcpyHostToDevice,
                            S.stream));
  HIPCHK(c0, hipMemcpyAsync(S.work.p, all.data(), all.size() * sizeof(int4), hipMemcpyHostToDevice, S.stream));
  HIPCHK(c0, hipStreamSynchronize(S.stream));
  // capture the sweep
  std::vector<int> cur, prev, out;
  roles(S.degree, cur, prev, out, S.final_buf);
  HIPCHK(c0, hipStreamBeginCapture(S.stream, hipStreamCaptureModeThreadLocal));
  if (sizeof(T) == 4)
    for (int m : S.members) {
      Item &it = items[m];
      copy_cols_launch<double, float>(it.X, it.ld, it.c->fbuf[0].as<float>(), it.o->nblock, it.c->mesh.n_dof,
                                      it.o->nblock, S.stream);
    }
  int lerr = 0;
  for (int k = 0; k < S.degree; ++k)
    for (size_t g = 0; g < S.groups.size(); ++g)
      lerr |= hx_cells_batch_launch<T>(S.groups[g].first, S.probs.template as<BatchProblem<T>>(), S.work.template as<int4>() + S.goff[g],
                                       S.gcnt[g], k, cur[k], prev[k], out[k], S.stream);
  for (size_t m = 0; m < S.members.size(); ++m) {
    Item &it = items[S.members[m]];
    const BatchProblem<T> &P = hp[m];
    if (sizeof(T) == 4)
      copy_cols_launch<float, double>((const float *)P.buf[S.final_buf], P.ld[S.final_buf], it.X, it.ld,
                                      it.c->mesh.n_dof, it.o->nblock, S.stream);
    else if (S.final_buf != 0)
      copy_cols_launch<double, double>((const double *)P.buf[S.final_buf], P.ld[S.final_buf], it.X, it.ld,
                                       it.c->mesh.n_dof, it.o->nblock, S.stream);
  }
  hipError_t ce = hipStreamEndCapture(S.stream, &S.graph);
  if (ce != hipSuccess) return fail(c0, CHFSI_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  if (lerr) return fail(c0, CHFSI_ERR_ARG, "batch: no cell kernel for a problem's degree");
  HIPCHK(c0, hipGraphInstantiate(&S.exec, S.graph, nullptr, nullptr, 0));
  return 0;
}

template <typename T>
int run_batch(std::vector<Item> &items, int degree, int max_iter, int threads, chfsi_ctx *c0) {
  Sweep<T> S;
  S.degree = degree;
  HIPCHK(c0, hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      if (s) (void)hipStreamDestroy(s);
    }
  } sg{S.stream};
  // start: CholGS + RR of every start block
  int st = parallel_for((int)items.size(), threads, [&](int i) {
    Item &it = items[i];
    if (int r = set_dev(it.c)) return r;
    int passes = 0;
    if (int r = orth_robust(it.c, it.X, it.ld, it.o->nblock, 0, &passes)) return r;
    if (int r = rr_impl(it.c, it.X, it.ld, it.o->nblock, it.c->HX.as<double>(), it.o->nblock, it.evals, it.resid,
                        nullptr))
      return r;
    it.res = max_wanted(it);
    it.active = it.res > it.o->tol && it.o->max_iter > 0;
    return 0;
  });
  if (st) return st;
  std::vector<int> last_members;
  std::vector<T> hcoef;
  for (int pass = 0; pass < max_iter; ++pass) {
    std::vector<int> members;
    for (auto &it : items)
      if (it.active) members.push_back(it.idx);
    if (members.empty()) break;
    if (members != last_members) {
      if (int r = build_sweep<T>(S, items, c0)) return r;
      last_members = members;
    }
    // per-problem coefficients of the normalised recursion
    hcoef.assign((size_t)3 * degree * members.size(), T(0));
    for (size_t m = 0; m < members.size(); ++m) {
      Item &it = items[members[m]];
      const int nb = it.o->nblock;
      const double a = it.evals[nb - 1], a0 = it.evals[0], b = it.c->ub;
      if (!(a0 < a && a < b)) return fail(c0, CHFSI_ERR_NONFINITE, "batch: Ritz values outside the filter bounds");
      const double cc = 0.5 * (a + b), e = 0.5 * (b - a), xi0 = (a0 - cc) / e;
      double rho = 1.0 / xi0;
      T *tc = hcoef.data() + (size_t)3 * degree * m;
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
        tc[3 * k] = (T)s1;
        tc[3 * k + 1] = (T)s2;
        tc[3 * k + 2] = (T)cc;
      }
    }
    HIPCHK(c0, hipMemcpyAsync(S.coef.p, hcoef.data(), hcoef.size() * sizeof(T), hipMemcpyHostToDevice, S.stream));
    hipEvent_t e0, e1;
    HIPCHK(c0, hipEventCreate(&e0));
    HIPCHK(c0, hipEventCreate(&e1));
    (void)hipEventRecord(e0, S.stream);
    HIPCHK(c0, hipGraphLaunch(S.exec, S.stream));
    (void)hipEventRecord(e1, S.stream);
    HIPCHK(c0, hipStreamSynchronize(S.stream));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // CholGS + RR per problem
    st = parallel_for((int)members.size(), threads, [&](int m) {
      Item &it = items[members[m]];
      if (int r = set_dev(it.c)) return r;
      int passes = 0;
      if (int r = orth_robust(it.c, it.X, it.ld, it.o->nblock, it.o->mixed_cholgs ? 1 : 0, &passes)) return r;
      if (int r = rr_impl(it.c, it.X, it.ld, it.o->nblock, it.c->HX.as<double>(), it.o->nblock, it.evals, it.resid,
                          nullptr))
        return r;
      it.rep.iters++;
      it.rep.t_filter += ms * 1e-3;
      it.rep.dofvecs += it.c->mesh.n_dof * (int64_t)it.o->nblock * (degree + 1);
      it.res = max_wanted(it);
      it.active = it.res > it.o->tol && it.rep.iters < it.o->max_iter;
      return 0;
    });
    if (st) return st;
    if (c0->verbose) {
      int na = 0;
      double worst = 0;
      for (auto &it : items) {
        na += it.active;
        worst = std::max(worst, it.res);
      }
      std::fprintf(stderr, "[chfsi] batch pass %d: %zu problems swept (%.3f ms), %d still active, max residual %.3e\n",
                   pass, members.size(), ms, na, worst);
      std::fflush(stderr);
    }
  }
  return 0;
}

}  // namespace

extern "C" int chfsi_solve_batch(chfsi_ctx *const *ctxs, int n, const chfsi_opts *opts, double *const *X,
                                 const int64_t *ld, double *const *evals, double *const *resid, chfsi_report *reps) {
  if (!ctxs || n < 1 || !opts || !X || !ld || !evals || !resid) return CHFSI_ERR_ARG;
  chfsi_ctx *c0 = ctxs[0];
  if (!c0) return CHFSI_ERR_ARG;
  const int degree = opts[0].degree;
  chfsi_prec prec = opts[0].n_ladder > 0 ? opts[0].ladder[0] : CHFSI_FP64;
  int max_iter = 0;
  std::vector<Item> items(n);
  for (int i = 0; i < n; ++i) {
    chfsi_ctx *c = ctxs[i];
    const chfsi_opts *o = &opts[i];
    if (!c) return fail(c0, CHFSI_ERR_ARG, "batch: null context");
    if (c->device != c0->device) return fail(c0, CHFSI_ERR_ARG, "batch: contexts on different devices");
    if (int r = check_block(c, X[i], ld[i], o->nblock)) return fail(c0, r, std::string("batch: ") + c->err);
    if (o->nstates < 1 || o->nstates > o->nblock || o->degree != degree || degree < 1 || o->max_iter < 0 ||
        !(o->tol > 0) || !evals[i] || !resid[i] || o->nblock > c->mesh.n_dof)
      return fail(c0, CHFSI_ERR_ARG, "batch: invalid options (every problem needs the same degree)");
    const chfsi_prec p = o->n_ladder > 0 ? o->ladder[0] : CHFSI_FP64;
    if (p != prec || (p != CHFSI_FP64 && p != CHFSI_FP32))
      return fail(c0, CHFSI_ERR_ARG, "batch: one filter precision (FP64 or FP32) for every problem");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(c0, CHFSI_ERR_ARG, "batch: a context appears twice");
    if (int r = ensure_small(c, o->nblock)) return r;
    const size_t bytes = (size_t)c->mesh.n_dof * o->nblock * (prec == CHFSI_FP64 ? 8 : 4);
    for (int k = (prec == CHFSI_FP64 ? 1 : 0); k < 3; ++k) HIPCHK(c, c->fbuf[k].ensure(bytes));
    HIPCHK(c, c->HX.ensure((size_t)c->mesh.n_dof * o->nblock * sizeof(double)));
    Item &it = items[i];
    it.idx = i;
    it.c = c;
    it.o = o;
    it.X = X[i];
    it.ld = ld[i];
    it.evals = evals[i];
    it.resid = resid[i];
    std::memset(&it.rep, 0, sizeof it.rep);
    max_iter = std::max(max_iter, o->max_iter);
  }
  if (int r = set_dev(c0)) return r;
  const int threads = 8;
  int st = prec == CHFSI_FP64 ? run_batch<double>(items, degree, max_iter, threads, c0)
                              : run_batch<float>(items, degree, max_iter, threads, c0);
  if (st) return st;
  int worst = CHFSI_OK;
  for (auto &it : items) {
    it.rep.max_resid = it.res;
    it.rep.status = it.res <= it.o->tol ? CHFSI_OK : CHFSI_WARN_NOT_CONVERGED;
    if (it.rep.status != CHFSI_OK) worst = CHFSI_WARN_NOT_CONVERGED;
    if (reps) reps[it.idx] = it.rep;
  }
  return worst;
}
