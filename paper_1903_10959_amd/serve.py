"""Served stream of solve requests on one GPU (host control over the C ABI).

A request is one SCF-like sequence: a problem drawn from the batched-workload
size distribution, solved `solves` times; solve 1 starts from a seeded block,
solve s > 1 warm-starts from solve s-1's vectors (kept on the device) with the
potential perturbed by 1 % seeded noise (the paper reuses the previous
wavefunctions as the starting guess, Sec. 3.3).

Scheduling: requests arrive by a seeded Poisson process.  A request is
admitted when a slot is free and its device footprint (``chfsi_footprint_bytes``
plus its blocks) fits the HBM budget next to the requests already running;
otherwise it waits in arrival order.  Each slot is a host thread with its own
library contexts and HIP stream, so admitted requests run concurrently on the
device; a slot keeps the contexts of its last meshes (mesh tables stay on the
device).  Every number a request produces depends only on the request: alone
or in the mix, its results are the same.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time

import numpy as np

from . import Context, footprint_bytes


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float             # seconds after the stream starts
    problem: object            # workload.Problem
    footprint: int = 0
    admitted: float = 0.0
    done: float = 0.0
    solve_times: list = dataclasses.field(default_factory=list)
    iters: list = dataclasses.field(default_factory=list)
    evals: list = dataclasses.field(default_factory=list)
    converged: bool = True


def make_stream(n_requests: int, rate: float, seed: int = 5, sizes=None):
    """Seeded Poisson arrivals; problems drawn from the batched-workload sizes."""
    import workload

    rng = np.random.Generator(np.random.PCG64(seed))
    pool = sizes if sizes is not None else workload.batch_problems(64, 4)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        out.append(Request(i, t, pool[int(rng.integers(0, len(pool)))]))
    return out


class _Slot:
    """One concurrent lane: a stream and a small cache of contexts by mesh."""

    def __init__(self, device: int, cache: int = 2):
        import torch

        self.stream = torch.cuda.Stream(device)
        self.device = device
        self.cache = collections.OrderedDict()
        self.cache_size = cache

    def context(self, prob):
        key = (prob.L, prob.n_el, prob.p)
        if key in self.cache:
            self.cache.move_to_end(key)
            return self.cache[key]
        while len(self.cache) >= self.cache_size:
            _, old = self.cache.popitem(last=False)
            old.close()
        c = Context(self.device, stream=self.stream).set_mesh(prob.L, prob.n_el, prob.p)
        self.cache[key] = c
        return c

    def close(self):
        for c in self.cache.values():
            c.close()
        self.cache.clear()


_V0_CACHE = {}
_V0_LOCK = threading.Lock()


def _base_potential(prob, ctx):
    """Unperturbed potential of a problem, evaluated once per problem."""
    import workload

    with _V0_LOCK:
        v = _V0_CACHE.get(prob.name)
    if v is None:
        v = workload.eval_wells(workload.problem_wells(prob), ctx.dof_coords())
        with _V0_LOCK:
            _V0_CACHE[prob.name] = v
    return v


def run_request(slot: _Slot, req: Request, solves: int, tol: float, degree: int, ladder, stream_seed: int,
                t0: float):
    import torch

    import workload

    prob = req.problem
    with torch.cuda.stream(slot.stream):
        ctx = slot.context(prob)
        V0 = _base_potential(prob, ctx)
        X = workload.start_block_device(prob.n_dof, prob.nblock, prob.x0_seed, device=f"cuda:{slot.device}")
        for s in range(solves):
            ts = time.time()
            V = V0 if s == 0 else workload.perturbed(V0, (stream_seed, req.rid, s))
            ctx.set_potential(V)
            out = ctx.solve(X, prob.nstates, degree, tol, max_iter=400, ladder=ladder)
            slot.stream.synchronize()
            req.solve_times.append(time.time() - ts)
            req.iters.append(out["iters"])
            req.evals.append(out["evals"][:prob.nstates].copy())
            req.converged = req.converged and out["converged"]
    req.done = time.time() - t0


def serve(requests, slots: int = 8, hbm_budget: float = 160e9, solves: int = 5, tol: float = 1e-6,
          degree: int = 20, ladder=("fp32", "fp64"), stream_seed: int = 5, device: int = 0, log=None,
          realtime: bool = True):
    """Run the stream; returns the requests with timings filled in.
    realtime=False admits every request at t = 0 (offline replay)."""
    for r in requests:
        r.footprint = footprint_bytes(r.problem.n_el, r.problem.p, r.problem.nblock, 0, ladder[0]) \
            + r.problem.n_dof * r.problem.nblock * 8
        if r.footprint > hbm_budget:
            raise ValueError(f"request {r.rid} needs {r.footprint} B, above the HBM budget")
    lanes = [_Slot(device) for _ in range(slots)]
    free = queue.Queue()
    for ln in lanes:
        free.put(ln)
    lock = threading.Lock()
    in_use = [0.0]
    cond = threading.Condition(lock)
    threads = []
    errors = []
    t0 = time.time()

    def finish(slot, req):
        try:
            run_request(slot, req, solves, tol, degree, ladder, stream_seed, t0)
        except Exception as exc:  # surfaced after the run
            errors.append((req.rid, exc))
        finally:
            with cond:
                in_use[0] -= req.footprint
                cond.notify_all()
            free.put(slot)
            if log:
                log(f"request {req.rid} done at {req.done:.2f} s ({sum(req.solve_times):.2f} s of solves)")

    for req in sorted(requests, key=lambda r: r.arrival):
        if realtime:
            wait = req.arrival - (time.time() - t0)
            if wait > 0:
                time.sleep(wait)
        slot = free.get()                     # a slot frees up
        with cond:                            # and the memory fits
            while in_use[0] + req.footprint > hbm_budget:
                cond.wait()
            in_use[0] += req.footprint
        req.admitted = time.time() - t0
        th = threading.Thread(target=finish, args=(slot, req))
        th.start()
        threads.append(th)
    for th in threads:
        th.join()
    for ln in lanes:
        ln.close()
    if errors:
        raise RuntimeError(f"{len(errors)} requests failed; first: {errors[0]}")
    return requests


def latency_stats(requests, wall: float):
    e2e = np.array([r.done - r.arrival for r in requests])
    qd = np.array([r.admitted - r.arrival for r in requests])
    per_solve = np.array([t for r in requests for t in r.solve_times])
    span = max(r.arrival for r in requests) - min(r.arrival for r in requests)
    return {
        "requests": len(requests),
        "offered_rate_per_s": (len(requests) - 1) / span if span > 0 else None,
        "achieved_rate_per_s": len(requests) / wall,
        "e2e_p50_s": float(np.percentile(e2e, 50)), "e2e_p99_s": float(np.percentile(e2e, 99)),
        "queue_p50_s": float(np.percentile(qd, 50)), "queue_p99_s": float(np.percentile(qd, 99)),
        "solve_p50_s": float(np.percentile(per_solve, 50)), "solve_p99_s": float(np.percentile(per_solve, 99)),
        "all_converged": all(r.converged for r in requests),
    }
