"""Pins of the oracle's spectrum-splitting Rayleigh-Ritz and electron density
(Alg. 4, Alg. 5, eqs. elecDens and elecDensSP), CPU only."""
import numpy as np
import pytest

from oracle import chfsi, density, fem
import workload


def _small_problem():
    prob = workload.PROBLEMS["small"]
    V = workload.eval_wells(workload.problem_wells(prob), fem.dof_coords(prob.L, prob.n_el, prob.p))
    H = fem.htilde_csr(prob.L, prob.n_el, prob.p, V)
    _, M = fem.assemble(prob.L, prob.n_el, prob.p)
    return prob, H, M


def test_fermi_dirac_symmetry_and_midpoint():
    mu, sigma = -0.3, 1.6e-3
    d = np.linspace(-0.05, 0.05, 41)
    f = density.fermi_dirac(mu + d, mu, sigma)
    np.testing.assert_allclose(f + density.fermi_dirac(mu - d, mu, sigma), 1.0, rtol=0, atol=1e-15)
    assert density.fermi_dirac(mu, mu, sigma) == 0.5
    assert np.all(np.diff(f) <= 0)                 # decreasing in the energy
    assert density.fermi_dirac(mu + 10.0, mu, sigma) == 0.0   # no overflow warning path


def test_fermi_level_two_levels_is_the_midpoint():
    """Two fractional levels sharing one electron pair: f(e1) + f(e2) = 1 holds
    exactly at mu = (e1 + e2)/2 by the symmetry above."""
    e = np.array([-0.412, -0.377])
    mu = density.fermi_level(e, n_oc=7, n_electrons=2 * (7 + 1), sigma=3e-3)
    assert abs(mu - e.mean()) < 1e-13


def test_fermi_level_symmetric_spectrum():
    rng = np.random.default_rng(3)
    mu0 = 0.25
    d = rng.uniform(0.001, 0.05, 9)
    e = np.sort(np.concatenate([mu0 - d, mu0 + d]))
    mu = density.fermi_level(e, n_oc=40, n_electrons=2 * (40 + 9), sigma=0.01)
    assert abs(mu - mu0) < 1e-13
    # and the count it solves for
    assert abs(density.electron_count(e, 40, mu, 0.01) - 98) < 1e-12


def test_fermi_level_rejects_impossible_counts():
    e = np.array([0.1, 0.2, 0.3])
    for ne in (2 * 4, 2 * 4 - 1e-300, 2 * 7, 2 * 9):
        with pytest.raises(ValueError):
            density.fermi_level(e, n_oc=4, n_electrons=ne, sigma=0.01)


def test_split_rr_fp64_is_the_top_of_the_full_rr():
    prob, H, _ = _small_problem()
    ap = lambda X: H @ X
    X = chfsi.cholgs(workload.start_block(H.shape[0], 40, 11))
    Xr, _, D, res = chfsi.rayleigh_ritz(ap, X)
    Xfr, Dfr, rfr = density.rayleigh_ritz_split(ap, X, 8)
    np.testing.assert_allclose(Dfr, D[32:], rtol=0, atol=1e-12)
    np.testing.assert_allclose(rfr, res[32:], rtol=1e-8, atol=1e-12)
    sgn = np.sign(np.sum(Xfr * Xr[:, 32:], axis=0))
    np.testing.assert_allclose(Xfr * sgn, Xr[:, 32:], rtol=0, atol=1e-10)


def _density_setup(nb=40, n_fr=8, sigma=0.02):
    prob, H, M = _small_problem()
    ap = lambda X: H @ X
    X = chfsi.cholgs(workload.start_block(H.shape[0], nb, 12))
    Xfr, Dfr, _ = density.rayleigh_ritz_split(ap, X, n_fr)
    n_oc = nb - n_fr
    ne = 2 * (n_oc + 0.37 * n_fr)
    mu = density.fermi_level(Dfr, n_oc, ne, sigma)
    return H, M, X, Xfr, Dfr, n_oc, ne, mu, sigma


def test_density_integrates_to_the_electron_count():
    """sum_j M_jj rho_j = 2 sum_i f_i ||x_i||^2 = N_e for orthonormal X (the
    constraint of Sec. 2.1 that fixes mu)."""
    H, M, X, Xfr, Dfr, n_oc, ne, mu, sigma = _density_setup()
    rho = density.density_split(X, Xfr, Dfr, mu, sigma, 1.0 / np.sqrt(M))
    assert abs(np.sum(M * rho) - ne) < 1e-11 * ne
    assert np.all(rho > -1e-14)


def test_split_density_equals_full_rotation_density():
    """eq. elecDensSP and eq. elecDens give the same density: X X^T = X Q Q^T X^T."""
    H, M, X, Xfr, Dfr, n_oc, ne, mu, sigma = _density_setup()
    Xr, _, D, _ = chfsi.rayleigh_ritz(lambda Y: H @ Y, X)
    minv = 1.0 / np.sqrt(M)
    r_split = density.density_split(X, Xfr, Dfr, mu, sigma, minv)
    r_full = density.density_full(Xr, D, n_oc, mu, sigma, minv)
    np.testing.assert_allclose(r_split, r_full, rtol=0, atol=1e-12 * np.max(np.abs(r_full)))


def test_cell_level_formula_matches_nodal_density_on_every_cell():
    """eq. elecDensSums through each cell's Lagrange basis at its GLL nodes
    equals the nodal form at the node's DoF (and 0 at Dirichlet nodes)."""
    L, n_el, p = 6.0, 2, 3
    V = workload.eval_wells(workload.draw_wells(2, L, 5, (1.0, 2.0), (0.5, 1.0)), fem.dof_coords(L, n_el, p))
    H = fem.htilde_csr(L, n_el, p, V)
    _, M = fem.assemble(L, n_el, p)
    minv = 1.0 / np.sqrt(M)
    X = chfsi.cholgs(workload.start_block(H.shape[0], 10, 13))
    Xr, _, D, _ = chfsi.rayleigh_ritz(lambda Y: H @ Y, X)
    n_oc = 7
    mu = density.fermi_level(D[n_oc:], n_oc, 2 * (n_oc + 1.5), 0.05)
    occ = np.ones(10)
    occ[n_oc:] = density.fermi_dirac(D[n_oc:], mu, 0.05)
    cells = density.density_cellwise(L, n_el, p, Xr, occ, minv)
    nodal = density.density_full(Xr, D, n_oc, mu, 0.05, minv)
    cmap = fem.cell_dof_map(n_el, p)
    for e in range(cmap.shape[0]):
        live = cmap[e] >= 0
        np.testing.assert_allclose(cells[e, live], nodal[cmap[e, live]], rtol=1e-12, atol=1e-15)
        assert np.all(np.abs(cells[e, ~live]) < 1e-15)


def test_box_ground_state_density_is_the_product_of_1d_densities():
    """V = 0: the ground state of the 3D operator (dense eigh) is separable, and
    with half occupancy (N_e = 1, mu = lambda_0) its density is the product of
    three 1D densities u(x)^2 / m(x), m the assembled 1D GLL mass."""
    L, n_el, p = 9.0, 3, 4
    n = n_el * p - 1
    H = fem.htilde_csr(L, n_el, p, np.zeros(n ** 3))
    _, M = fem.assemble(L, n_el, p)
    lam, U = chfsi.eig_dense(H)
    x0 = U[:, :1]
    mu = density.fermi_level(lam[:1], 0, 1.0, 1e-3)
    assert abs(mu - lam[0]) < 1e-12
    # one state, fractionally occupied: basis and rotated vector coincide
    rho = density.density_split(x0, x0, lam[:1], mu, 1e-3, 1.0 / np.sqrt(M))
    # 1D: eigenvector of the 1D operator, mass from the GLL weights
    a, u = np.linalg.eigh(fem.operator_1d(L, n_el, p))
    _, w = fem.gll(p)
    h = L / n_el
    m1 = np.zeros(n_el * p + 1)
    for e in range(n_el):
        m1[e * p:e * p + p + 1] += 0.5 * h * w
    m1 = m1[1:-1]
    g = u[:, 0] ** 2 / m1
    expect = np.kron(g, np.kron(g, g))             # dof = I + n J + n^2 K
    np.testing.assert_allclose(rho, expect, rtol=1e-9, atol=1e-12 * np.max(expect))
    np.testing.assert_allclose(M, np.kron(m1, np.kron(m1, m1)), rtol=1e-13)


@pytest.mark.parametrize("L,n_el,p", [(9.0, 3, 4), (6.0, 2, 3), (10.0, 4, 5)])
def test_kron_mass_equals_assembled_mass(L, n_el, p):
    _, M = fem.assemble(L, n_el, p)
    np.testing.assert_allclose(fem.mass_diag_kron(L, n_el, p), M, rtol=1e-14)
