"""Served stream on the GPU: results are the same alone and in the mix, and
every warm-started solve of a perturbed potential matches the dense
eigensolve of that potential."""
import numpy as np
import pytest

from oracle import fem
import workload

pytestmark = pytest.mark.gpu


def _pool():
    mk = lambda i, n_el, p, N: workload.Problem(f"srv{i}", 2.5 * n_el, n_el, p, N, 20, 0, 700 + i, 750 + i, 4,
                                                (1.0, 3.0), (0.3, 0.6))
    return [mk(0, 4, 4, 16), mk(1, 3, 5, 24), mk(2, 4, 5, 20), mk(3, 3, 6, 12)]


def test_served_results_alone_equal_results_in_the_mix():
    from paper_1903_10959_amd import serve as S
    pool = _pool()
    mix = S.make_stream(10, 1000.0, seed=11, sizes=pool)
    S.serve(mix, solves=3, tol=1e-6, realtime=False)
    for r in mix:
        assert r.converged and len(r.evals) == 3
    for r in mix[:3]:
        alone = S.Request(r.rid, 0.0, r.problem)
        S.serve([alone], solves=3, tol=1e-6, realtime=False)
        for a, b in zip(alone.evals, r.evals):
            np.testing.assert_array_equal(a, b)
        assert alone.iters == r.iters


def test_served_solves_match_dense_eigh_of_each_perturbed_potential():
    """Solve s of request r runs on V_0 (1 + 0.01 xi), xi seeded by
    (stream seed, r, s), warm-started from solve s - 1: its wanted
    eigenvalues equal those of the dense eigensolve of that potential's
    operator to the served tolerance (a residual of 1e-6 Ha bounds each
    Ritz value's distance to the spectrum)."""
    from paper_1903_10959_amd import serve as S
    small = [pr for pr in _pool() if pr.n_dof <= 3375]
    reqs = S.make_stream(5, 1000.0, seed=13, sizes=small)
    tol = 1e-6
    S.serve(reqs, solves=3, tol=tol, realtime=False, stream_seed=5)
    for r in reqs:
        pr = r.problem
        assert r.converged and len(r.evals) == 3
        V0 = workload.eval_wells(workload.problem_wells(pr), fem.dof_coords(pr.L, pr.n_el, pr.p))
        for s, ev in enumerate(r.evals):
            V = V0 if s == 0 else workload.perturbed(V0, (5, r.rid, s))
            ref = np.linalg.eigvalsh(fem.htilde_csr(pr.L, pr.n_el, pr.p, V).toarray())[:pr.nstates]
            assert np.max(np.abs(ev - ref)) <= tol, (r.rid, s, np.max(np.abs(ev - ref)))


def test_admission_respects_the_hbm_budget():
    from paper_1903_10959_amd import serve as S
    pool = _pool()
    reqs = S.make_stream(4, 1000.0, seed=12, sizes=pool)
    big = max(S.request_footprint(p) for p in pool)
    # a budget that fits one request at a time serialises the stream (idle
    # contexts are freed to make room)
    S.serve(reqs, hbm_budget=big * 1.01, solves=1, tol=1e-4, realtime=False)
    spans = sorted((r.admitted, r.done) for r in reqs)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0 - 1e-3
