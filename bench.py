"""Benchmark: ChFSI H.X throughput (DoF-vecs/s) on one MI355X.

One step = one pass of the whole hot path over the 1,128-vector block of the
32^3-cell, degree-5 workload (4,019,679 DoFs, 64 seeded Gaussian wells, 1,024
wanted states + 104 guard states): Chebyshev filter of degree 30 in blocks of
128 vectors, CholGS, Rayleigh-Ritz (one more Htilde application, projection,
Jacobi eigensolve, rotation, residuals).  value = Htilde applications in the
step x n_dof / step time (inputs resident in HBM).  --workload large_p6 runs
the 24^3-cell, degree-6 workload (568 vectors) instead.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3}          # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                              # GB/s


def host_cpu():
    """CPU model and physical core count of this host (from /proc/cpuinfo)."""
    model, cores = "unknown", set()
    phys = core = None
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name":
                model = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                core = v
            elif not k and phys is not None:
                cores.add((phys, core))
                phys = core = None
    except OSError:
        pass
    return model, (len(cores) or os.cpu_count() or 1)


def cpu_baseline(prob, ncols: int, nrows: int = 16384):
    """The oracle, as it stands, timed on a bounded sample of one ChFSI
    iteration and scaled by each part's own cost model to the whole block:
    * filter: the degree-m filter on `ncols` of the vectors (its cost per
      vector does not depend on the block), scaled by N_b / ncols, plus one
      more application per vector for Rayleigh-Ritz;
    * CholGS and the Rayleigh-Ritz products at the full block width N_b on
      `nrows` rows of the block (their cost is linear in the rows), scaled by
      n_dof / nrows; the N_b x N_b factorisations and eigensolve inside them
      are timed on their own and counted once."""
    import numpy as np
    import scipy.linalg as sla
    from threadpoolctl import threadpool_info

    import workload
    from oracle import chfsi as och
    from oracle import fem

    nb = prob.nblock
    xyz = fem.dof_coords(prob.L, prob.n_el, prob.p)
    V = workload.eval_wells(workload.problem_wells(prob), xyz)
    A = fem.operator_1d(prob.L, prob.n_el, prob.p)
    apply = lambda X: fem.apply_kron(A, V, X)
    b = fem.upper_bound(A, V)
    X = och.cholgs(workload.start_block(prob.n_dof, ncols, prob.x0_seed))
    _, _, D, _ = och.rayleigh_ritz(apply, X)
    t0 = time.time()
    och.cheb_filter_scaled(apply, X, prob.degree, float(D[-1]), b, float(D[0]))
    t_filter = time.time() - t0
    per_apply = t_filter / (prob.degree * ncols)
    Xs = workload.start_block(nrows, nb, prob.x0_seed + 1)
    t0 = time.time()
    Xs = och.cholgs(Xs)
    t_chol = time.time() - t0
    t0 = time.time()
    och.rayleigh_ritz(lambda Y: Y * 1.0, Xs)
    t_rr = time.time() - t0
    S = Xs.T @ Xs + np.eye(nb)
    t0 = time.time()
    Lc = np.linalg.cholesky(S)
    sla.solve_triangular(Lc, np.eye(nb), lower=True)
    np.linalg.eigh(S)
    t_dense = time.time() - t0
    t_iter = ((prob.degree + 1) * nb * per_apply + max(t_chol + t_rr - t_dense, 0.0) * prob.n_dof / nrows
              + t_dense)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    model, phys = host_cpu()
    dofvecs = prob.n_dof * nb * (prob.degree + 1)
    sampled = t_filter + t_chol + t_rr + t_dense
    return {"value": dofvecs / t_iter, "unit": "DoF-vecs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one ChFSI iteration of the Kronecker-form FP64 oracle, estimated from {sampled:.1f} s "
                      f"of timed parts: degree-{prob.degree} filter on {ncols} of {nb} vectors (x {nb / ncols:.1f}), "
                      f"CholGS + Rayleigh-Ritz at width {nb} on {nrows} of {prob.n_dof} rows "
                      f"(x {prob.n_dof / nrows:.1f}), N_b^3 factorisations once; whole iteration "
                      f"{t_iter:.0f} s",
            "seconds_estimated": t_iter, "cpu_model": model, "physical_cores": phys}


def profiled_traffic(tag: str, sources=("hx.hip", "common.hpp")):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary profiles/<tag>.md, or None when that summary is missing or
    the kernel source changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{tag}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256_16"):
            k, v = line.split(":", 1)
            vals[k.strip()] = (v.split() or [""])[0]     # a trailing "(files)" note is not part of it
    csrc = os.path.join(ROOT, "paper_1903_10959_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in sources)
    if vals.get("kernel_source_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def batch_throughput(args):
    """The batched workload: 64 independent problems (n_el 4..12, p 4..7,
    16..256 states) through chfsi_solve_batch for a fixed number of passes
    (FP32 filter of degree 20, FP64 CholGS/RR), against the same passes solved
    one problem at a time with chfsi_solve."""
    import numpy as np
    import torch

    import paper_1903_10959_amd as P
    import workload

    probs = workload.batch_problems(64, 4)
    passes = args.steps
    dev = torch.device("cuda:0")
    ctxs, Xs, Ns = [], [], []
    t0 = time.time()
    for pr in probs:
        c = P.Context(0, stream=torch.cuda.Stream(dev)).set_mesh(pr.L, pr.n_el, pr.p)
        c.set_potential(workload.eval_wells(workload.problem_wells(pr), c.dof_coords()))
        ctxs.append(c)
        Xs.append(workload.start_block_device(pr.n_dof, pr.nblock, pr.x0_seed, device=dev))
        Ns.append(pr.nstates)
    torch.cuda.synchronize()
    # autotuned cell-kernel tile per degree (FP32 filter): timed once per p on
    # a scratch copy of one problem's block, then set on every context of that p
    from paper_1903_10959_amd import autotune as AT

    tiles = {}
    t_tune = time.time()
    for i, pr in enumerate(probs):
        if pr.p not in tiles:
            c = ctxs[i]
            scratch = Xs[i].clone()
            b = c.upper_bound
            tiles[pr.p] = AT.tune_tile_variant(c, scratch, (0.5 * b, b, -50.0), prec="fp32", refresh=True)
            del scratch
        ctxs[i].set_tile_variant(tiles[pr.p])
    # cells per work-group per (degree, block size): blocks of few columns pad
    # fewer MFMA columns with more cells per tile
    cpts = {}
    for i, pr in enumerate(probs):
        key = (pr.p, pr.nblock)
        if key not in cpts:
            c = ctxs[i]
            scratch = Xs[i].clone()
            b = c.upper_bound
            cpts[key] = AT.tune_cells_per_tile(c, scratch, (0.5 * b, b, -50.0), prec="fp32", refresh=True)
            del scratch
        ctxs[i].set_cells_per_tile(cpts[key])
    torch.cuda.synchronize()
    print(f"[bench] batch: tile variants per degree {tiles}, cells per tile per (p, N_b) {cpts} "
          f"(tuned in {time.time() - t_tune:.1f} s)", file=sys.stderr, flush=True)
    tot_dofs = sum(pr.n_dof for pr in probs)
    print(f"[bench] batch: {len(probs)} problems, {tot_dofs} DoFs in all, setup {time.time() - t0:.1f} s",
          file=sys.stderr, flush=True)
    starts = [X.clone() for X in Xs]
    # one pass first: build, graph capture and first-touch allocations
    P.solve_batch(ctxs, [X.clone() for X in Xs], Ns, 20, 1e-30, max_iter=1, prec="fp32")
    torch.cuda.synchronize()
    t0 = time.time()
    res = P.solve_batch(ctxs, Xs, Ns, 20, 1e-30, max_iter=passes, prec="fp32")
    torch.cuda.synchronize()
    t_batch = time.time() - t0
    dofvecs = sum(pr.n_dof * pr.nblock * (20 * r["iters"] + r["iters"] + 1) for pr, r in zip(probs, res))
    print(f"[bench] batch: {passes} passes in {t_batch:.2f} s", file=sys.stderr, flush=True)
    t0 = time.time()
    for c, X0, pr in zip(ctxs, starts, probs):
        c.solve(X0, pr.nstates, 20, 1e-30, max_iter=passes, ladder=("fp32",))
    torch.cuda.synchronize()
    t_seq = time.time() - t0
    print(f"[bench] one at a time: {t_seq:.2f} s", file=sys.stderr, flush=True)
    out = {"metric": "batched ChFSI H.X DoF-vecs/s (64 independent problems, FP32 filter, FP64 CholGS/RR)",
           "value": dofvecs / t_batch, "unit": "DoF-vecs/s", "n_gpus": 1, "steps": passes, "warmup": 1,
           "ms_per_step": t_batch / passes * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32-filter/f64", "data": "synthetic",
           "config": {"workload": "batch: 64 problems, n_el in 4..12, p in 4..7, N in 16..256, L = 2.5 n_el, "
                                  f"{tot_dofs} DoFs in all, Chebyshev degree 20"},
           "one_at_a_time_seconds": t_seq, "batch_seconds": t_batch, "speedup_vs_one_at_a_time": t_seq / t_batch,
           "tile_variant_per_degree": {str(k): v for k, v in sorted(tiles.items())},
           "cells_per_tile_per_degree_and_block": {f"p{k[0]}/nb{k[1]}": v for k, v in sorted(cpts.items())}}
    print(json.dumps(out), flush=True)
    for c in ctxs:
        c.close()


def served_stream(args):
    """Served stream: seeded Poisson arrivals of solve requests (sizes of the
    batched workload), 5 warm-started solves each with a 1 % perturbed
    potential, HBM-footprint admission, continuous batching; p50/p99 latency."""
    import torch

    from paper_1903_10959_amd import serve as S

    lt = [float(v) for v in args.ladder_tol.split(",")] if args.ladder_tol else None
    rates = [float(r) for r in args.rates.split(",")] if args.rates else [args.rate]
    curve = []
    for rate in rates:
        reqs = S.make_stream(args.requests, rate, seed=5)
        t0 = time.time()
        S.serve(reqs, hbm_budget=args.hbm_budget, solves=5, tol=args.tol, degree=20, ladder=("fp32", "fp64"),
                ladder_tol=lt, log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        wall = time.time() - t0
        st = S.latency_stats(reqs, wall)
        st["offered_rate_setting_per_s"] = rate
        st["throughput_dofvecs_per_s"] = sum(r.problem.n_dof * r.problem.nblock * (20 + 1) * sum(r.iters)
                                             for r in reqs) / wall
        st["wall_s"] = wall
        curve.append(st)
        print(f"[bench] serve at {rate}/s: achieved {st['achieved_rate_per_s']:.3f}/s, e2e p50 "
              f"{st['e2e_p50_s']:.2f} s p99 {st['e2e_p99_s']:.2f} s, queue p99 {st['queue_p99_s']:.2f} s",
              file=sys.stderr, flush=True)
    st = curve[-1]
    out = {"metric": "served ChFSI stream: p99 end-to-end request latency (5 warm-started solves per request)",
           "value": st["e2e_p99_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
           "dtype": "fp32-filter->f64", "data": "synthetic",
           "config": {"workload": f"served: {args.requests} requests per offered rate, Poisson arrivals, sizes of "
                                  f"the batched workload, 5 solves each to residual {args.tol} Ha, continuous "
                                  f"batching, HBM budget {args.hbm_budget / 1e9:.0f} GB",
                      "rates_per_s": rates},
           "latency": st, "curve": curve, "ladder_tol": lt}
    print(json.dumps(out), flush=True)


def time_to_solution(args, prob, bw):
    """Wall time of chfsi_solve from the seeded start block until every wanted
    residual is <= tol (|Ritz value - exact eigenvalue| <= residual for a
    symmetric operator), FP64 path vs the mixed path (the filter precision
    ladder, default BF16 -> FP32 -> FP64, each rung left when the residual
    stalls or falls below its precision's floor; mixed-precision CholGS)."""
    os.environ.setdefault("CHFSI_VERBOSE", "1")   # the solve prints one line per pass
    import numpy as np
    import torch

    import paper_1903_10959_amd as P
    import workload

    dev = torch.device("cuda:0")
    ctx = P.Context(0).set_mesh(prob.L, prob.n_el, prob.p)
    V = workload.eval_wells(workload.problem_wells(prob), ctx.dof_coords())
    ctx.set_potential(V)
    runs = {}
    ladder = tuple(args.ladder.split(","))
    variants = [("fp64", dict(ladder=("fp64",), mixed_cholgs=False)),
                ("mixed", dict(ladder=ladder, mixed_cholgs=True))]
    for name, kw in variants:
        X = workload.start_block_device(prob.n_dof, prob.nblock, prob.x0_seed, device=dev)
        torch.cuda.synchronize()
        t0 = time.time()
        out = ctx.solve(X, prob.nstates, prob.degree, args.tol, max_iter=args.max_iter, block_width=bw, **kw)
        torch.cuda.synchronize()
        dt = time.time() - t0
        runs[name] = dict(seconds=dt, iters=out["iters"], converged=out["converged"], rung=out["rung"],
                          max_resid=out["max_resid"], t_filter=out["t_filter"], t_cholgs=out["t_cholgs"],
                          t_rr=out["t_rr"], evals_head=[float(x) for x in out["evals"][:4]],
                          evals=out["evals"][:prob.nstates].tolist())
        print(f"[bench] tts {name}: {dt:.2f} s, {out['iters']} passes, converged={out['converged']}, "
              f"max resid {out['max_resid']:.2e}", file=sys.stderr, flush=True)
        del X
        torch.cuda.empty_cache()
    e64 = np.array(runs["fp64"].pop("evals"))
    emx = np.array(runs["mixed"].pop("evals"))
    res = {
        "metric": "ChFSI time to eigenpairs with residual <= 1e-6 Ha (FP64 path vs mixed path)",
        "value": runs["fp64"]["seconds"] / runs["mixed"]["seconds"],
        "unit": "speedup (FP64 time / mixed time)",
        "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "data": "synthetic",
        "dtype": "f64 vs " + "->".join(ladder) + " filter ladder/mixed-CholGS",
        "config": {"workload": workload.fmt_problem(prob), "tol_Ha": args.tol, "filter_block": bw},
        "fp64": runs["fp64"], "mixed": runs["mixed"],
        "max_abs_eval_diff_mixed_vs_fp64": float(np.max(np.abs(e64 - emx))),
    }
    print(json.dumps(res), flush=True)
    ctx.close()


def kpoint_solve(args, prob):
    """ChFSI at a k-point (complex Hermitian Bloch operator, FP64) on the
    periodic cell with the workload's element size and degree: whole passes
    (complex filter of the workload's degree, Hermitian CholGS, Hermitian
    Rayleigh-Ritz) on a block of N = 256 complex states (N_b = 288), timed
    after warm-up passes.  value = complex DoF-vecs per second over the
    passes (n_dof x N_b x (degree + 1) per pass)."""
    import numpy as np
    import torch

    import paper_1903_10959_amd as P
    import workload

    dev = torch.device("cuda:0")
    ctx = P.Context(0).set_mesh(prob.L, prob.n_el, prob.p, periodic=True)
    ctx.set_potential(workload.eval_wells(workload.problem_wells(prob), ctx.dof_coords()))
    k = (0.05, 0.11, -0.08)
    ctx.set_kpoint(k)
    N = 256
    nb = workload.block_size(N)
    g = torch.Generator(device=dev).manual_seed(prob.x0_seed)
    X = torch.randn((ctx.n_dof, nb), dtype=torch.complex128, device=dev, generator=g)
    ctx.solve_complex(X, N, prob.degree, 1e-30, max_iter=max(1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.time()
    out = ctx.solve_complex(X, N, prob.degree, 1e-30, max_iter=args.steps)
    torch.cuda.synchronize()
    dt = time.time() - t0
    passes = out["iters"]
    dv = ctx.n_dof * nb * (prob.degree + 1) * passes / dt
    res = {"metric": "ChFSI at a k-point: complex DoF-vecs/s over whole passes (filter + CholGS + RR), FP64",
           "value": dv, "unit": "complex DoF-vecs/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
           "data": "synthetic", "dtype": "f64 (complex128)",
           "config": {"workload": f"periodic [0,{prob.L})^3, {prob.n_el}^3 cells, p={prob.p}, {ctx.n_dof} DoFs, "
                                  f"k={list(k)}, N={N}, N_b={nb}, Chebyshev degree {prob.degree}",
                      "passes": passes},
           "s_per_pass": dt / passes, "t_filter_s": out["t_filter"], "t_cholgs_s": out["t_cholgs"],
           "t_rr_s": out["t_rr"], "max_wanted_resid": out["max_resid"],
           "upper_bound_k": ctx.upper_bound_k}
    print(json.dumps(res), flush=True)
    del X
    ctx.close()


def rr_split_compare(args, prob):
    """Rayleigh-Ritz cost: the full procedure (all pairs, full rotation) against
    spectrum splitting with the mixed-precision projection (Alg. 4:
    N_fr = 15 % of N largest pairs, partial rotation), on the same block."""
    import numpy as np
    import torch

    import paper_1903_10959_amd as P
    import workload

    dev = torch.device("cuda:0")
    ctx = P.Context(0).set_mesh(prob.L, prob.n_el, prob.p)
    ctx.set_potential(workload.eval_wells(workload.problem_wells(prob), ctx.dof_coords()))
    X0 = workload.start_block_device(prob.n_dof, prob.nblock, prob.x0_seed, device=dev)
    ctx.orthonormalize(X0)
    ev0, _ = ctx.rayleigh_ritz(X0)
    # the block Rayleigh-Ritz sees inside a ChFSI pass: filtered, then
    # orthonormalised (not yet a Ritz basis of its own span)
    ctx.chebyshev_filter(X0, prob.degree, float(ev0[-1]), ctx.upper_bound, float(ev0[0]),
                         block_width=prob.block_width)
    ctx.orthonormalize(X0)
    n_fr = max(1, int(round(0.15 * prob.nstates)))
    nb = prob.nblock
    times = {"full": [], "split_mixed": [], "split_fp64": []}
    out = {}
    for rep in range(args.steps + 1):
        for name in times:
            X = X0.clone()
            torch.cuda.synchronize()
            t0 = time.time()
            if name == "full":
                ev, rs = ctx.rayleigh_ritz(X)
                out[name] = ev[nb - n_fr:]
            else:
                ev, rs = ctx.rayleigh_ritz_split(X, n_fr, mixed=(name == "split_mixed"))
                out[name] = ev
            torch.cuda.synchronize()
            if rep > 0:
                times[name].append(time.time() - t0)
            del X
    ms = {k: 1e3 * float(np.median(v)) for k, v in times.items()}
    res = {"metric": "Rayleigh-Ritz wall time: full vs spectrum splitting with mixed-precision projection",
           "value": ms["full"] / ms["split_mixed"], "unit": "speedup (full / split-mixed)", "n_gpus": 1,
           "higher_is_better": True, "vs_baseline": None, "data": "synthetic", "dtype": "f64 / f32-outside-fr-fr",
           "config": {"workload": workload.fmt_problem(prob), "n_fr": n_fr, "N_b": nb},
           "ms": ms, "steps": args.steps,
           "max_abs_fr_eval_diff_mixed_vs_full": float(np.max(np.abs(out["split_mixed"] - out["full"]))),
           "max_abs_fr_eval_diff_fp64_split_vs_full": float(np.max(np.abs(out["split_fp64"] - out["full"])))}
    print(json.dumps(res), flush=True)
    ctx.close()


def density_bench(args, prob):
    """Electron density (Alg. 5) on the block: spectrum-splitting RR into a
    separate X Q_fr (Alg. 4, mixed projection), the Fermi level, and the
    nodal density kernel, timed with HIP events on the context's stream (the
    torch current stream).  Roofline: HBM, algorithmic bytes per launch =
    n_dof (8 (N_b + N_fr) + 16): read X and X Q_fr rows, M^-1/2, write rho."""
    import numpy as np
    import torch

    import paper_1903_10959_amd as P
    import workload

    dev = torch.device("cuda:0")
    ctx = P.Context(0).set_mesh(prob.L, prob.n_el, prob.p)
    ctx.set_potential(workload.eval_wells(workload.problem_wells(prob), ctx.dof_coords()))
    X = workload.start_block_device(prob.n_dof, prob.nblock, prob.x0_seed, device=dev)
    ctx.orthonormalize(X)
    ev0, _ = ctx.rayleigh_ritz(X)
    # one filter pass, so the Ritz values (and mu) sit in the low spectrum
    ctx.chebyshev_filter(X, prob.degree, float(ev0[-1]), ctx.upper_bound, float(ev0[0]),
                         block_width=prob.block_width)
    ctx.orthonormalize(X)
    nb = prob.nblock
    n_fr = max(1, int(round(0.15 * prob.nstates)))
    n_oc = nb - n_fr
    Xfr = torch.empty((prob.n_dof, n_fr), dtype=torch.float64, device=dev)
    t_rr = []
    for rep in range(args.steps + 1):
        torch.cuda.synchronize()
        t0 = time.time()
        ev, _ = ctx.rayleigh_ritz_split(X, n_fr, mixed=True, Xfr=Xfr)
        torch.cuda.synchronize()
        if rep > 0:
            t_rr.append(time.time() - t0)
    sigma = 1.58e-3                                   # k_B T at 500 K
    ne = 2 * (n_oc + 0.5 * n_fr)
    t0 = time.perf_counter()
    mu = P.fermi_level(ev, n_oc, ne, sigma)
    t_mu = time.perf_counter() - t0
    rho = torch.empty(prob.n_dof, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        ctx.density(X, Xfr, ev, mu, sigma, rho=rho)
    reps = max(1, 10 * args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.density(X, Xfr, ev, mu, sigma, rho=rho)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = prob.n_dof * (8 * (nb + n_fr) + 16)
    gbs = nbytes / (ms * 1e-3) / 1e9
    res = {"metric": "electron density (Alg. 5) HBM throughput", "value": gbs, "unit": "GB/s", "n_gpus": 1,
           "higher_is_better": True, "vs_baseline": None, "data": "synthetic", "dtype": "f64",
           "config": {"workload": workload.fmt_problem(prob), "N_b": nb, "n_fr": n_fr, "sigma_Ha": sigma},
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                        "traffic": profiled_traffic(f"density_{prob.name}", ("dense.hip",)),
                        "kernel": "density_kernel", "bytes_per_launch": nbytes,
                        "avg_launch_ms": ms},
           "ms": {"split_rr_out_of_place": 1e3 * float(np.median(t_rr)), "fermi_level": 1e3 * t_mu,
                  "density": ms},
           "mu_Ha": mu, "steps": args.steps}
    print(json.dumps(res), flush=True)
    ctx.close()


def kpoint_bench(args, prob):
    """Complex Bloch operator (Sec. 2.1 eq. ksproblemPer) on the periodic cell
    with the workload's element size and degree: Y = Htilde_k X for a complex
    block of 64 vectors (one filter block of 128 real columns), timed with HIP
    events on the context's stream.  Roofline: FP64 MFMA, algorithmic flops =
    8 n_loc^2 per cell per complex vector (A Xr + B Xi and A Xi - B Xr)."""
    import torch

    import numpy as np

    import paper_1903_10959_amd as P
    import workload

    dev = torch.device("cuda:0")
    ctx = P.Context(0).set_mesh(prob.L, prob.n_el, prob.p, periodic=True)
    ctx.set_potential(workload.eval_wells(workload.problem_wells(prob), ctx.dof_coords()))
    k = (0.05, 0.11, -0.08)
    ctx.set_kpoint(k)
    nc = 64
    g = torch.Generator(device=dev).manual_seed(prob.x0_seed)
    X = torch.randn((ctx.n_dof, nc), dtype=torch.complex128, device=dev, generator=g)
    Y = torch.empty_like(X)
    for _ in range(max(1, args.warmup)):
        ctx.apply_complex(X, Y)
    reps = max(1, 10 * args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.apply_complex(X, Y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 8.0 * ctx.n_loc ** 2 * ctx.n_cells * nc
    tf = flops / (ms * 1e-3) / 1e12
    dv = ctx.n_dof * nc / (ms * 1e-3)
    del X, Y
    # a k-point group (2 x 2 x 2 Monkhorst-Pack set) on a batch-sized periodic
    # mesh: one launch per colour for all k-points vs one context per k-point
    Lg, neg, pg = 20.0, 8, 5
    kk = [(2 * np.pi / Lg) * np.array([sx, sy, sz]) / 4 for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)]
    grp = P.Context(0).set_mesh(Lg, neg, pg, periodic=True)
    Vg = workload.eval_wells(workload.draw_wells(8, Lg, 4), grp.dof_coords())
    grp.set_potential(Vg)
    grp.set_kpoints(kk)
    Xg = torch.randn((len(kk), grp.n_dof, nc), dtype=torch.complex128, device=dev, generator=g)
    Yg = torch.empty_like(Xg)
    singles = []
    for kv in kk:
        cs = P.Context(0).set_mesh(Lg, neg, pg, periodic=True)
        cs.set_potential(Vg)
        cs.set_kpoint(kv)
        singles.append(cs)

    def timed(fn, n=reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    ms_group = timed(lambda: grp.apply_complex_kpoints(Xg, Yg))
    ms_single = timed(lambda: [cs.apply_complex(Xg[i], Yg[i]) for i, cs in enumerate(singles)])
    for cs in singles:
        cs.close()
    grp.close()
    res = {"metric": "complex Bloch operator Htilde_k X DoF-vecs/s (periodic cell, FP64)", "value": dv,
           "unit": "complex DoF-vecs/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
           "data": "synthetic", "dtype": "f64 (complex128)",
           "config": {"workload": f"periodic [0,{prob.L})^3, {prob.n_el}^3 cells, p={prob.p}, {ctx.n_dof} DoFs, "
                                  f"k={list(k)}, {nc} complex vectors", "steps": args.steps},
           "roofline": {"bound": "mfma", "achieved": tf, "peak": 78.6, "unit": "TFLOP/s", "frac": tf / 78.6,
                        "traffic": profiled_traffic(f"hx_cells_cplx_periodic_p{prob.p}"),
                        "kernel": "hx_cells_cplx_kernel", "avg_apply_ms": ms, "launches_per_apply": 8,
                        "flop_per_cell_complex_vec": 8 * ctx.n_loc ** 2},
           "kpoint_group": {"mesh": f"periodic [0,{Lg})^3, {neg}^3 cells, p={pg}", "nk": len(kk),
                            "complex_vectors_per_k": nc, "ms_group": ms_group, "ms_one_context_per_k": ms_single,
                            "speedup": ms_single / ms_group}}
    print(json.dumps(res), flush=True)
    ctx.close()


def poisson_bench(args, prob):
    """Electrostatics (eq. phiTotDiscreteSolve, Dirichlet) on the workload's
    mesh: Jacobi-PCG to a 1e-10 relative residual for the density of the
    workload's wells plus point charges at two nodes.  Roofline of the
    matrix-free product: HBM, algorithmic bytes = 16 per DoF (read x, write y).
    A whole CG iteration moves 80 algorithmic bytes per DoF: the product reads
    p and writes q, the update reads r and q and writes r, the direction pass
    reads x, p and r and writes x and p (z = r / diag(A) is recomputed where it
    is used)."""
    import numpy as np
    import torch

    import paper_1903_10959_amd as P
    import workload

    dev = torch.device("cuda:0")
    ctx = P.Context(0).set_mesh(prob.L, prob.n_el, prob.p)
    rho = torch.from_numpy(-workload.eval_wells(workload.problem_wells(prob), ctx.dof_coords())).to(dev)
    charges = [(prob.n_dof // 3, -6.0), (2 * prob.n_dof // 3, -4.0)]
    times, its = [], []
    for rep in range(args.steps + 1):
        phi = torch.zeros_like(rho)
        torch.cuda.synchronize()
        t0 = time.time()
        out = ctx.poisson_solve(rho, phi, charges=charges, tol=1e-10)
        torch.cuda.synchronize()
        if rep > 0:
            times.append(time.time() - t0)
            its.append(out["iters"])
    x = torch.randn(prob.n_dof, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ctx.poisson_apply(x, y)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.poisson_apply(x, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 16.0 * prob.n_dof / (ms * 1e-3) / 1e9
    t = float(np.median(times))
    res = {"metric": "Poisson solve (Jacobi-PCG to 1e-10) time", "value": t, "unit": "s", "n_gpus": 1,
           "higher_is_better": False, "vs_baseline": None, "data": "synthetic", "dtype": "f64",
           "config": {"workload": f"Dirichlet [0,{prob.L}]^3, {prob.n_el}^3 cells, p={prob.p}, {prob.n_dof} DoFs; "
                                  f"density of the workload's 64 wells + 2 point charges", "steps": args.steps},
           "iterations": its[-1], "ms_per_iteration": 1e3 * t / max(1, its[-1]), "rel_resid": out["rel_resid"],
           "iteration_hbm_gbs": 80.0 * prob.n_dof * max(1, its[-1]) / t / 1e9,
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                        "traffic": profiled_traffic(f"poisson_{prob.name}", ("poisson.hip",)),
                        "kernel": "poisson_stencil_kernel", "avg_launch_ms": ms,
                        "bytes_per_launch": 16 * prob.n_dof}}
    print(json.dumps(res), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large_p5")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16", "bf16x3"])
    ap.add_argument("--mixed-cholgs", action="store_true")
    ap.add_argument("--block-width", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=16)
    ap.add_argument("--mode", default="step",
                    choices=["step", "tts", "rr", "density", "kpoint", "ksolve", "poisson"],
                    help="step: throughput of whole ChFSI iterations (default); tts: time to solution; "
                         "rr: Rayleigh-Ritz full vs spectrum splitting; density: electron density (Alg. 5); "
                         "kpoint: complex Bloch operator on the periodic cell; ksolve: ChFSI at a k-point; "
                         "poisson: electrostatics (Jacobi-PCG)")
    ap.add_argument("--tol", type=float, default=1e-6, help="tts: residual tolerance (Ha)")
    ap.add_argument("--max-iter", type=int, default=200)
    ap.add_argument("--requests", type=int, default=48, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: Poisson arrival rate per second")
    ap.add_argument("--rates", default="", help="serve: comma-separated offered rates (one run each; the last is "
                                                "the headline); default --rate")
    ap.add_argument("--hbm-budget", type=float, default=160e9, help="serve: device bytes for admitted requests")
    ap.add_argument("--ladder", default="bf16,fp32,fp64", help="tts: filter precisions of the mixed path's ladder")
    ap.add_argument("--ladder-tol", default="",
                    help="serve: residual (Ha) ending each precision rung, comma separated (default 4 u b per rung)")
    ap.add_argument("--calib-bytes", type=int, default=0,
                    help="first run a plain elementwise copy (y = x * 1) of this many bytes, three times: "
                         "the reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; there is no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1903_10959_amd as P
    import workload

    if args.workload == "batch":
        return batch_throughput(args)
    if args.workload == "serve":
        return served_stream(args)
    prob = workload.PROBLEMS[args.workload]
    bw = args.block_width or prob.block_width
    dev = torch.device("cuda:0")
    if args.calib_bytes > 0:
        xc = torch.ones(args.calib_bytes // 8, dtype=torch.float64, device=dev)
        yc = torch.empty_like(xc)
        for _ in range(3):
            torch.mul(xc, 1.0, out=yc)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {args.calib_bytes} bytes read + written, 3 launches", file=sys.stderr,
              flush=True)
        del xc, yc
    print(f"[bench] {workload.fmt_problem(prob)} B={bw} prec={args.prec} on {torch.cuda.get_device_name(0)}",
          file=sys.stderr, flush=True)
    if args.mode == "tts":
        return time_to_solution(args, prob, bw)
    if args.mode == "density":
        return density_bench(args, prob)
    if args.mode == "kpoint":
        return kpoint_bench(args, prob)
    if args.mode == "ksolve":
        return kpoint_solve(args, prob)
    if args.mode == "poisson":
        return poisson_bench(args, prob)
    if args.mode == "rr":
        return rr_split_compare(args, prob)
    ctx = P.Context(0).set_mesh(prob.L, prob.n_el, prob.p)
    V = workload.eval_wells(workload.problem_wells(prob), ctx.dof_coords())
    ctx.set_potential(V)
    b = ctx.upper_bound
    nb = prob.nblock
    X = workload.start_block_device(prob.n_dof, nb, prob.x0_seed, device=dev)
    ctx.orthonormalize(X, mixed=args.mixed_cholgs)
    ev, rs = ctx.rayleigh_ritz(X)
    torch.cuda.synchronize()
    print(f"[bench] setup done; initial Ritz range [{ev[0]:.4f}, {ev[-1]:.4f}], b={b:.2f}", file=sys.stderr,
          flush=True)

    def step(ev):
        ctx.chebyshev_filter(X, prob.degree, float(ev[-1]), b, float(ev[0]), prec=args.prec, block_width=bw)
        ctx.orthonormalize(X, mixed=args.mixed_cholgs)
        return ctx.rayleigh_ritz(X)

    for w in range(args.warmup):
        t0 = time.time()
        ev, rs = step(ev)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w}: {time.time() - t0:.3f} s, max wanted resid {np.max(rs[:prob.nstates]):.3e}",
              file=sys.stderr, flush=True)

    # timed region: the cell-product launches are bracketed by HIP events --
    # in FP64 every launch of the step (the filter's and the Rayleigh-Ritz
    # applications, all the same kernel), in a reduced precision the filter's
    # launches only (the Rayleigh-Ritz applications run the FP64 kernel)
    ctx.set_timing(True)
    ctx.reset_timing()
    t_filter = 0.0
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(args.steps):
        ts = time.time()
        ctx.chebyshev_filter(X, prob.degree, float(ev[-1]), b, float(ev[0]), prec=args.prec, block_width=bw)
        t_filter += time.time() - ts   # filter returns after its finiteness check (synchronised)
        if args.prec != "fp64":
            ctx.set_timing(False)
        ctx.orthonormalize(X, mixed=args.mixed_cholgs)
        ev, rs = ctx.rayleigh_ritz(X)
        ctx.set_timing(True)
        print(f"[bench] step {k}: max wanted resid {np.max(rs[:prob.nstates]):.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.time() - t0
    tim = ctx.filter_timing()
    ctx.set_timing(False)

    ms_step = dt / args.steps * 1e3
    dofvecs_step = prob.n_dof * nb * (prob.degree + 1)
    value = dofvecs_step / (dt / args.steps)
    n_loc = (prob.p + 1) ** 3
    n_cells = prob.n_el ** 3
    avg_launch_ms = tim["ms"] / max(tim["launches"], 1)
    if args.prec in ("fp64", "fp32"):
        # MFMA-bound: the method's dense cell products, 2 n_loc^2 flops per cell-vector
        flops = 2.0 * n_loc * n_loc * tim["cell_vecs"]
        achieved = flops / (tim["ms"] * 1e-3) / 1e12
        peak, bound, unit = PEAK[args.prec], "mfma", "TFLOP/s"
        kname = f"hx_cells_kernel<{'double' if args.prec == 'fp64' else 'float'},{(n_loc + 15) // 16 * 16}>"
    else:
        # HBM-bound: 3 x 4 B of FP32 recursion state per DoF-vec (read X_k, X_k-1, write X_k+1)
        dofvecs = tim["cell_vecs"] * prob.n_dof / n_cells
        achieved = 12.0 * dofvecs / (tim["ms"] * 1e-3) / 1e9
        peak, bound, unit = HBM_PEAK, "hbm", "GB/s"
        kname = f"hx_cells_bf16_kernel<{(n_loc + 31) // 32 * 32},{'true' if args.prec == 'bf16x3' else 'false'}>"
    out = {
        "metric": "ChFSI H.X DoF-vecs/s (whole ChFSI iteration: filter + CholGS + RR)",
        "value": value,
        "unit": "DoF-vecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" and not args.mixed_cholgs else f"{args.prec}-filter/f64",
        "data": "synthetic",
        "config": {"workload": f"{prob.name}: [0,{prob.L:g}]^3, {prob.n_el}^3 cells, GLL p={prob.p}, "
                               f"{prob.n_dof} DoFs, {prob.n_wells} seeded Gaussian wells, N={prob.nstates}, "
                               f"N_b={nb}, Chebyshev degree {prob.degree}, filter block {bw}",
                   "filter_precision": args.prec, "mixed_cholgs": bool(args.mixed_cholgs)},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak,
                     "traffic": profiled_traffic(f"hx_cells_{prob.name}_{args.prec}"),
                     "kernel": kname,
                     "launches": tim["launches"], "avg_launch_ms": avg_launch_ms,
                     "flop_per_cell_vec": 2 * n_loc * n_loc},
        "filter_dofvecs_per_s": prob.n_dof * nb * prob.degree / (t_filter / args.steps),
        "max_wanted_resid": float(np.max(rs[:prob.nstates])),
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host (bounded sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_cols)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
