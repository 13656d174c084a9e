"""GPU parity of the matrix-free Poisson operator and its Jacobi-PCG solve
(Sec. 2.4 eq. phiTotDiscreteSolve, Dirichlet) against the oracle."""
import numpy as np
import pytest

import paper_1903_10959_amd as P
from oracle import fem, poisson
import workload

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


@pytest.mark.parametrize("L,n_el,p", [(6.0, 2, 1), (6.0, 2, 3), (8.0, 3, 4), (10.0, 4, 6), (7.0, 2, 7),
                                      (30.0, 12, 6), (26.0, 13, 5)])   # 71^3, 64^3: several ragged tiles
def test_poisson_apply_matches_oracle(L, n_el, p):
    c = P.Context(0).set_mesh(L, n_el, p)
    A, _ = poisson.poisson_matrix(L, n_el, p)
    x = np.random.default_rng(n_el * 10 + p).standard_normal(c.n_dof)
    y = c.poisson_apply(_t(x)).cpu().numpy()
    yo = A @ x
    assert np.max(np.abs(y - yo)) < 1e-13 * np.max(np.abs(yo))
    c.close()


def test_poisson_solve_matches_oracle_with_point_charges():
    L, n_el, p = 8.0, 3, 4
    c = P.Context(0).set_mesh(L, n_el, p)
    xyz = fem.dof_coords(L, n_el, p)
    rho = -workload.eval_wells(workload.draw_wells(3, L, 6, (0.5, 1.0), (0.5, 1.0)), xyz)   # positive density
    charges = [(17, -2.0), (1000, -1.0), (17, 0.5)]
    out = c.poisson_solve(_t(rho), charges=charges, tol=1e-12)
    assert out["converged"] and out["rel_resid"] <= 1e-12
    A, M = poisson.poisson_matrix(L, n_el, p)
    f = poisson.load_vector(M, rho, [d for d, _ in charges], [q for _, q in charges])
    phi_o = poisson.solve(L, n_el, p, rho, [d for d, _ in charges], [q for _, q in charges])
    phi = out["phi"].cpu().numpy()
    assert np.max(np.abs(phi - phi_o)) < 1e-10 * np.max(np.abs(phi_o))
    # the same algorithm: the device records the iteration at which its own
    # test first held (sums in another order can move that by one at most)
    _, it_o, _ = poisson.jacobi_pcg(A, f, tol=1e-12)
    assert abs(out["iters"] - it_o) <= 1, (out["iters"], it_o)
    c.close()


def test_poisson_manufactured_solution():
    L, n_el, p = 6.0, 3, 7
    c = P.Context(0).set_mesh(L, n_el, p)
    phi_x, rho = poisson.manufactured(L, fem.dof_coords(L, n_el, p))
    out = c.poisson_solve(_t(rho), tol=1e-13)
    assert np.max(np.abs(out["phi"].cpu().numpy() - phi_x)) < 1e-9
    c.close()


def test_poisson_warm_start_and_argument_checks():
    import torch
    L, n_el, p = 6.0, 2, 4
    c = P.Context(0).set_mesh(L, n_el, p)
    phi_x, rho = poisson.manufactured(L, fem.dof_coords(L, n_el, p))
    first = c.poisson_solve(_t(rho), tol=1e-12)
    again = c.poisson_solve(_t(rho), phi=first["phi"].clone(), tol=1e-12)
    assert again["iters"] <= 4                      # starts converged: at most one check interval
    with pytest.raises(P.ChfsiError):
        c.poisson_solve(_t(rho), charges=[(c.n_dof, 1.0)])
    c.close()
    cp = P.Context(0).set_mesh(L, n_el, p, periodic=True)
    with pytest.raises(P.ChfsiError):
        cp.poisson_solve(torch.zeros(cp.n_dof, dtype=torch.float64, device="cuda:0"))
    cp.close()


@pytest.mark.parametrize("L,n_el,p,cap", [(8.0, 3, 4, 1), (8.0, 3, 4, 2), (8.0, 3, 4, 7), (8.0, 3, 4, 19),
                                          (30.0, 12, 6, 5)])   # 71^3: two I-chunks, rows wrapping across waves
def test_poisson_iterates_follow_the_oracle_pcg_step_by_step(L, n_el, p, cap):
    """With the iteration cap below convergence, the solve stops after exactly
    `cap` iterations, reports non-convergence, and its iterate equals the
    oracle's Jacobi-PCG iterate after the same number of steps (the same
    recurrences; only the summation order differs) -- a check of alpha, beta
    and the direction update, not only of the converged answer.  The returned
    relative residual is that of the returned iterate."""
    c = P.Context(0).set_mesh(L, n_el, p)
    xyz = fem.dof_coords(L, n_el, p)
    rho = -workload.eval_wells(workload.draw_wells(3, L, 6, (0.5, 1.0), (0.5, 1.0)), xyz)
    out = c.poisson_solve(_t(rho), charges=[(17, -2.0)], tol=1e-14, max_iter=cap)
    assert not out["converged"] and out["iters"] == cap
    A, M = poisson.poisson_matrix(L, n_el, p)
    f = poisson.load_vector(M, rho, [17], [-2.0])
    x_o, it_o, hist = poisson.jacobi_pcg(A, f, tol=1e-14, max_iter=cap)
    assert it_o == cap
    phi = out["phi"].cpu().numpy()
    assert np.max(np.abs(phi - x_o)) < 1e-11 * np.max(np.abs(x_o))
    np.testing.assert_allclose(out["rel_resid"], np.linalg.norm(f - A @ phi) / np.linalg.norm(f), rtol=1e-8)
    c.close()
