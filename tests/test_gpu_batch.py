"""Batched solve (many independent problems in shared launches) on the GPU."""
import numpy as np
import pytest

from oracle import fem
import workload
from gpu_util import make_ctx, to_gpu, to_host

pytestmark = pytest.mark.gpu

SPECS = [(2, 4, 8), (3, 3, 16), (2, 5, 12), (2, 6, 20), (3, 4, 10), (1, 7, 6)]


def _problems():
    import torch
    out = []
    for i, (n_el, p, N) in enumerate(SPECS):
        L = 2.5 * n_el
        wells = workload.draw_wells(4, L, 900 + i, (1.0, 3.0), (0.2, 0.4))
        c, V = make_ctx(L, n_el, p, wells=wells)
        c2, _ = make_ctx(L, n_el, p, V=V)
        nb = workload.block_size(N)
        X0 = workload.start_block(c.n_dof, nb, 950 + i)
        ev = np.linalg.eigvalsh(fem.htilde_csr(L, n_el, p, V).toarray())
        out.append(dict(ctx=c, ctx_single=c2, X0=X0, N=N, nb=nb, ev=ev))
    return out


def test_batch_fp64_equals_single_solves_and_dense_eigh():
    import paper_1903_10959_amd as P
    probs = _problems()
    Xb = [to_gpu(p["X0"]) for p in probs]
    res = P.solve_batch([p["ctx"] for p in probs], Xb, [p["N"] for p in probs], 20, 1e-9, max_iter=300,
                        prec="fp64")
    for p, r, X in zip(probs, res, Xb):
        assert r["converged"], r
        N = p["N"]
        err = np.abs(r["evals"][:N] - p["ev"][:N]) / np.maximum(np.abs(p["ev"][:N]), 1.0)
        assert np.max(err) < 1e-10
        Xs = to_gpu(p["X0"])
        s = p["ctx_single"].solve(Xs, N, 20, 1e-9, max_iter=300, block_width=p["nb"])
        # same arithmetic per problem: identical results alone and in the batch
        assert s["iters"] == r["iters"]
        np.testing.assert_array_equal(s["evals"], r["evals"])
        np.testing.assert_array_equal(to_host(Xs), to_host(X))
    for p in probs:
        p["ctx"].close()
        p["ctx_single"].close()


def test_batch_fp32_filter_within_its_floor():
    import paper_1903_10959_amd as P
    probs = _problems()
    Xb = [to_gpu(p["X0"]) for p in probs]
    res = P.solve_batch([p["ctx"] for p in probs], Xb, [p["N"] for p in probs], 20, 1e-3, max_iter=300,
                        prec="fp32")
    for p, r in zip(probs, res):
        assert r["converged"], r
        N = p["N"]
        # residual 1e-3 bounds the eigenvalue error; second order makes it far smaller
        assert np.max(np.abs(r["evals"][:N] - p["ev"][:N])) < 1e-3
    for p in probs:
        p["ctx"].close()
        p["ctx_single"].close()
