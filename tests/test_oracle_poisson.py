"""Pins of the oracle's discrete Poisson problem (Sec. 2.4 eq.
phiTotDiscreteSolve, Dirichlet), CPU only."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import fem, poisson


def _1d(L, n_el, p):
    """Assembled 1D Laplacian stiffness and GLL mass on the interior nodes,
    from the reference matrices (independent of fem.assemble)."""
    h = L / n_el
    _, w = fem.gll(p)
    K1 = fem.stiffness_1d_ref(p)
    n1 = n_el * p + 1
    k = np.zeros((n1, n1))
    m = np.zeros(n1)
    for e in range(n_el):
        s = slice(e * p, e * p + p + 1)
        k[s, s] += (2.0 / h) * K1
        m[s] += (h / 2.0) * w
    return k[1:-1, 1:-1], m[1:-1]


def test_manufactured_solution_converges_spectrally():
    """phi = prod sin(pi x/L) with rho = 3 pi phi / (4 L^2): the FE solution at
    the nodes approaches phi as the degree rises (fixed mesh)."""
    L, n_el = 6.0, 3
    errs = []
    for p in (3, 5, 7):
        xyz = fem.dof_coords(L, n_el, p)
        phi, rho = poisson.manufactured(L, xyz)
        phi_h = poisson.solve(L, n_el, p, rho)
        errs.append(np.max(np.abs(phi_h - phi)))
    assert errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20, errs
    assert errs[2] < 1e-6, errs


def test_matrix_is_spd_kronecker_sum():
    L, n_el, p = 5.0, 2, 3
    A, M = poisson.poisson_matrix(L, n_el, p)
    k, m = _1d(L, n_el, p)
    Mm = np.diag(m)
    S = (np.kron(Mm, np.kron(Mm, k)) + np.kron(Mm, np.kron(k, Mm)) + np.kron(k, np.kron(Mm, Mm))) / (4 * np.pi)
    Ad = A.toarray()
    np.testing.assert_allclose(Ad, S, rtol=0, atol=1e-13 * np.abs(S).max())
    np.testing.assert_allclose(M, np.kron(m, np.kron(m, m)), rtol=1e-14)
    assert np.linalg.eigvalsh(Ad)[0] > 0


def test_jacobi_pcg_reaches_direct_solution():
    L, n_el, p = 8.0, 3, 4
    A, M = poisson.poisson_matrix(L, n_el, p)
    rng = np.random.default_rng(1)
    f = poisson.load_vector(M, rng.standard_normal(A.shape[0]), [10, 500], [-3.0, 2.0])
    x_direct = spla.spsolve(A.tocsc(), f)
    x, it, hist = poisson.jacobi_pcg(A, f, tol=1e-12)
    assert hist[-1] <= 1e-12 and it < A.shape[0]
    assert np.max(np.abs(x - x_direct)) < 1e-9 * np.max(np.abs(x_direct))


def test_point_charge_reciprocity():
    """The potential at node j of a unit charge on node i equals that at i of
    a unit charge on j (A symmetric), and charges superpose."""
    L, n_el, p = 6.0, 2, 4
    nd = (n_el * p - 1) ** 3
    i, j = 37, 211
    zero = np.zeros(nd)
    pi_ = poisson.solve(L, n_el, p, zero, [i], [1.0])
    pj = poisson.solve(L, n_el, p, zero, [j], [1.0])
    assert abs(pi_[j] - pj[i]) < 1e-13 * abs(pi_[j])
    both = poisson.solve(L, n_el, p, zero, [i, j], [2.0, -0.5])
    np.testing.assert_allclose(both, 2.0 * pi_ - 0.5 * pj, rtol=0, atol=1e-13 * np.abs(both).max())
