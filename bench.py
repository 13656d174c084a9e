"""Benchmark: ChFSI H.X throughput (DoF-vecs/s) on one MI355X.

One step = one pass of the whole hot path over the 568-vector block of the
24^3-cell, degree-6 workload (2,924,207 DoFs, 64 seeded Gaussian wells,
512 wanted states + 56 guard states): Chebyshev filter of degree 30 in
blocks of 128 vectors, CholGS, Rayleigh-Ritz (one more Htilde application,
projection, Jacobi eigensolve, two rotations, residuals).  value = Htilde
applications in the step x n_dof / step time (inputs resident in HBM).

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


def cpu_baseline(prob, ncols: int, budget_s: float = 30.0):
    """The oracle, as it stands, on a bounded sample: one ChFSI iteration
    (filter of the same degree + CholGS + RR) on `ncols` of the vectors."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import workload
    from oracle import chfsi as och
    from oracle import fem

    t0 = time.time()
    xyz = fem.dof_coords(prob.L, prob.n_el, prob.p)
    V = workload.eval_wells(workload.problem_wells(prob), xyz)
    A = fem.operator_1d(prob.L, prob.n_el, prob.p)
    apply = lambda X: fem.apply_kron(A, V, X)
    X = och.cholgs(workload.start_block(prob.n_dof, ncols, prob.x0_seed))
    X, _, D, _ = och.rayleigh_ritz(apply, X)
    b = fem.upper_bound(A, V)
    setup = time.time() - t0
    t0 = time.time()
    Z = och.cheb_filter_scaled(apply, X, prob.degree, float(D[-1]), b, float(D[0]))
    Z = och.cholgs(Z)
    och.rayleigh_ritz(apply, Z)
    dt = time.time() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    dofvecs = prob.n_dof * ncols * (prob.degree + 1)
    return {"value": dofvecs / dt, "unit": "DoF-vecs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one ChFSI iteration (degree-{prob.degree} filter + CholGS + RR) on {ncols} of "
                      f"{prob.nblock} vectors, Kronecker-form FP64 operator, {dt:.1f} s (setup {setup:.1f} s)",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large_p6")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--mixed-cholgs", action="store_true")
    ap.add_argument("--block-width", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=8)
    ap.add_argument("--calib-bytes", type=int, default=0,
                    help="first run a plain elementwise copy (y = x * 1) of this many bytes, three times: "
                         "the reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1903_10959_amd as P
    import workload

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

    # timed region: the filter's cell-product launches are bracketed by HIP events
    ctx.set_timing(True)
    ctx.reset_timing()
    t_filter = 0.0
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(args.steps):
        ts = time.time()
        ctx.chebyshev_filter(X, prob.degree, float(ev[-1]), b, float(ev[0]), prec=args.prec, block_width=bw)
        t_filter += time.time() - ts   # filter returns after its finiteness check (synchronised)
        ctx.orthonormalize(X, mixed=args.mixed_cholgs)
        ev, rs = ctx.rayleigh_ritz(X)
        print(f"[bench] step {k}: max wanted resid {np.max(rs[:prob.nstates]):.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.time() - t0
    tim = ctx.filter_timing()
    ctx.set_timing(False)

    ms_step = dt / args.steps * 1e3
    dofvecs_step = prob.n_dof * nb * (prob.degree + 1)
    value = dofvecs_step / (dt / args.steps)
    n_loc = (prob.p + 1) ** 3
    flops = 2.0 * n_loc * n_loc * tim["cell_vecs"]
    avg_launch_ms = tim["ms"] / max(tim["launches"], 1)
    achieved = flops / (tim["ms"] * 1e-3) / 1e12
    peak = PEAK[args.prec]
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
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": f"hx_cells_kernel<{'double' if args.prec == 'fp64' else 'float'},"
                               f"{(n_loc + 15) // 16 * 16}>",
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
