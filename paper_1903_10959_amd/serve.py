"""Served stream of solve requests on one GPU, with continuous batching.

A request is one SCF-like sequence: a problem drawn from the batched-workload
size distribution, solved `solves` times; solve 1 starts from a seeded block,
solve s > 1 warm-starts from solve s-1's vectors (kept on the device) with the
potential perturbed by 1 % seeded noise (the paper reuses the previous
wavefunctions as the starting guess, Sec. 3.3).

Scheduling (one engine loop over a ``BatchSession``): requests arrive by a
seeded Poisson process.  At every pass boundary the engine admits waiting
requests in arrival order while their device footprint (what a context in a
batch session holds, ``chfsi_batch_footprint_bytes``, plus the block) fits the
HBM budget next to the requests already running and the idle contexts kept
for reuse (charged with the bytes they hold; the least recently used are freed
when a request would not fit otherwise); an admitted request gets a context
(reused from a pool keyed by mesh, so mesh tables stay on the device) and its
solve joins the session's shared filter sweeps at the next pass.  A solve that
fails on its own (its report carries an error status) ends its request, which
is marked failed; the others go on.  A solve leaves the session when its wanted
residuals reach the tolerance; the request then starts its next warm solve
or, after the last one, releases its memory.  The arithmetic of a problem
does not depend on the other problems sharing its passes, so every result is
the same alone and in the mix.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np

from . import BatchSession, Context, batch_footprint_bytes


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float             # seconds after the stream starts
    problem: object            # workload.Problem
    footprint: int = 0
    admitted: float = -1.0
    done: float = -1.0
    solve_times: list = dataclasses.field(default_factory=list)
    iters: list = dataclasses.field(default_factory=list)
    evals: list = dataclasses.field(default_factory=list)
    converged: bool = True
    failed: bool = False       # a solve ended with an error status


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


class _ContextPool:
    """Idle contexts by mesh; each context has its own stream.  ``idle_bytes``
    is the device memory the idle contexts hold."""

    def __init__(self, device: int, idle_cap: int = 16):
        self.device = device
        self.idle = collections.OrderedDict()   # key -> [(ctx, bytes), ...]
        self.idle_cap = idle_cap
        self.n_idle = 0
        self.idle_bytes = 0

    def get(self, prob):
        import torch

        key = (prob.L, prob.n_el, prob.p)
        lst = self.idle.get(key)
        if lst:
            self.n_idle -= 1
            c, nb = lst.pop()
            self.idle_bytes -= nb
            if not lst:
                del self.idle[key]
            return c
        return Context(self.device, stream=torch.cuda.Stream(self.device)).set_mesh(prob.L, prob.n_el, prob.p)

    def put(self, prob, ctx):
        key = (prob.L, prob.n_el, prob.p)
        nb = ctx.device_bytes()
        self.idle.setdefault(key, []).append((ctx, nb))
        self.idle.move_to_end(key)
        self.n_idle += 1
        self.idle_bytes += nb
        while self.n_idle > self.idle_cap:
            self.evict_one()

    def evict_one(self) -> bool:
        """Free the least recently returned idle context; False if none."""
        if not self.idle:
            return False
        k, lst = next(iter(self.idle.items()))
        c, nb = lst.pop(0)
        c.close()
        self.idle_bytes -= nb
        self.n_idle -= 1
        if not lst:
            del self.idle[k]
        return True

    def close(self):
        for lst in self.idle.values():
            for c, _ in lst:
                c.close()
        self.idle.clear()
        self.n_idle = 0
        self.idle_bytes = 0


def request_footprint(prob) -> int:
    """Device bytes of one admitted request: its context in the batch session
    plus its block of vectors."""
    return batch_footprint_bytes(prob.n_el, prob.p, prob.nblock) + prob.n_dof * prob.nblock * 8


def serve(requests, hbm_budget: float = 160e9, solves: int = 5, tol: float = 1e-6, degree: int = 20,
          ladder=("fp32", "fp64"), stream_seed: int = 5, device: int = 0, log=None, realtime: bool = True,
          max_active: int = 256, ladder_tol=None):
    """Run the stream; returns the requests with timings filled in.
    realtime=False makes every request available at t = 0 (offline replay)."""
    import torch

    import workload

    for r in requests:
        r.footprint = request_footprint(r.problem)
        if r.footprint > hbm_budget:
            raise ValueError(f"request {r.rid} needs {r.footprint} B, above the HBM budget")
    order = sorted(requests, key=lambda r: r.arrival)
    pool = _ContextPool(device)
    sess = BatchSession(device)
    waiting = collections.deque()
    running = {}          # session id -> [request, ctx, X, V0, solve index, solve start]
    in_use = 0.0
    nxt = 0
    n_done = 0
    t0 = time.time()
    now = lambda: time.time() - t0

    def start_solve(entry, s):
        req, ctx, X, V0 = entry[0], entry[1], entry[2], entry[3]
        V = V0 if s == 0 else workload.perturbed(V0, (stream_seed, req.rid, s))
        ctx.set_potential(V)
        pid = sess.add(ctx, X, req.problem.nstates, degree, tol, max_iter=400, ladder=ladder, ladder_tol=ladder_tol)
        entry[4], entry[5] = s, time.time()
        running[pid] = entry

    try:
        while n_done < len(order):
            t = now()
            while nxt < len(order) and (not realtime or order[nxt].arrival <= t):
                waiting.append(order[nxt])
                nxt += 1
            # admission at the pass boundary; idle contexts count against the
            # budget and are freed (least recently used first) to make room
            while waiting and len(running) < max_active:
                need = waiting[0].footprint
                while in_use + pool.idle_bytes + need > hbm_budget and pool.evict_one():
                    pass
                if in_use + pool.idle_bytes + need > hbm_budget:
                    break
                req = waiting.popleft()
                req.admitted = now()
                ctx = pool.get(req.problem)
                # a reused context may hold more than the estimate (buffers only grow)
                req.footprint = max(need, ctx.device_bytes() + req.problem.n_dof * req.problem.nblock * 8)
                in_use += req.footprint
                X = workload.start_block_device(req.problem.n_dof, req.problem.nblock, req.problem.x0_seed,
                                                device=f"cuda:{device}")
                torch.cuda.synchronize(device)
                start_solve([req, ctx, X, _base_potential(req.problem, ctx), 0, 0.0], 0)
            if not running:
                if waiting and pool.idle_bytes == 0:
                    raise RuntimeError("a waiting request cannot be admitted (budget)")
                if nxt < len(order):
                    time.sleep(max(0.0, order[nxt].arrival - now()))
                continue
            _, finished = sess.step()
            for pid, res in finished:
                entry = running.pop(pid)
                req, ctx, X, V0, s, ts = entry
                req.solve_times.append(time.time() - ts)
                req.iters.append(res["iters"])
                req.evals.append(res["evals"][:req.problem.nstates].copy())
                req.converged = req.converged and res["converged"]
                if res["status"] < 0:
                    req.failed = True
                if s + 1 < solves and not req.failed:
                    start_solve(entry, s + 1)
                else:
                    req.done = now()
                    in_use -= req.footprint
                    pool.put(req.problem, ctx)
                    n_done += 1
                    if log:
                        log(f"request {req.rid} done at {req.done:.2f} s ({sum(req.solve_times):.2f} s of solves)")
    finally:
        sess.close()
        pool.close()
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
