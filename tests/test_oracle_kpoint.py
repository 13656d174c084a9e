"""Pins of the oracle's periodic k-point operator (Sec. 2.1 eq. ksproblemPer on
the GLL discretisation), CPU only."""
import numpy as np
import pytest

from oracle import fem, kpoint
import workload


@pytest.mark.parametrize("L,n_el,p", [(6.0, 2, 3), (5.0, 2, 4), (7.0, 4, 2)])
def test_derivative_matrices_antisymmetric_after_periodic_assembly(L, n_el, p):
    _, G, _ = kpoint.assemble_periodic(L, n_el, p)
    for g in G:
        assert abs(g + g.T).max() < 1e-13 * abs(g).max()


@pytest.mark.parametrize("p", [1, 2, 4, 6, 7])
def test_gll_derivative_factor_is_exact(p):
    """w_a' l_a'(xi_a') (the GLL rule) equals int l_a' l_a' dxi by Gauss-Legendre
    quadrature exact to degree 2(p+2)-1 >= 2p - 1."""
    xi, w = fem.gll(p)
    C1 = np.diag(w) @ fem.deriv_matrix(p)
    xg, wg = np.polynomial.legendre.leggauss(p + 2)
    Lg = fem.lagrange_eval(xi, xg)
    dLg = fem.lagrange_deriv_eval(xi, xg)
    exact = Lg.T @ (wg[:, None] * dLg)
    np.testing.assert_allclose(C1, exact, rtol=0, atol=1e-12 * np.abs(exact).max())


@pytest.mark.parametrize("p,h", [(2, 1.3), (4, 0.7)])
def test_cell_convection_against_3d_quadrature(p, h):
    """int N_j d_x N_l by the 3D GLL rule with the general Lagrange basis
    evaluated at every quadrature point (no tensor shortcut)."""
    xi, w = fem.gll(p)
    q = p + 1
    Lv = fem.lagrange_eval(xi, xi)
    dLv = fem.lagrange_deriv_eval(xi, xi)
    nl = q ** 3
    G = np.zeros((nl, nl))
    for cq in range(q):
        for bq in range(q):
            for aq in range(q):
                W = w[aq] * w[bq] * w[cq] * (h / 2) ** 3
                N = np.einsum("c,b,a->cba", Lv[cq], Lv[bq], Lv[aq]).reshape(-1)
                dN = (2.0 / h) * np.einsum("c,b,a->cba", Lv[cq], Lv[bq], dLv[aq]).reshape(-1)
                G += W * np.outer(N, dN)
    gx, _, _ = kpoint.cell_convection(p, h)
    np.testing.assert_allclose(gx, G, rtol=0, atol=1e-13 * np.abs(G).max())


def test_htilde_k_hermitian_and_kronecker_sum():
    L, n_el, p = 5.0, 2, 3
    k = np.array([0.31, -0.52, 0.11])
    n = n_el * p
    H = kpoint.htilde_k_csr(L, n_el, p, np.zeros(n ** 3), k).toarray()
    assert np.abs(H - H.conj().T).max() < 1e-13 * np.abs(H).max()
    A = [kpoint.operator_1d_periodic(L, n_el, p, kd) for kd in k]
    I = np.eye(n)
    S = np.kron(I, np.kron(I, A[0])) + np.kron(I, np.kron(A[1], I)) + np.kron(A[2], np.kron(I, I))
    np.testing.assert_allclose(H, S, rtol=0, atol=1e-12 * np.abs(S).max())


@pytest.mark.parametrize("k", [0.0, 0.37, -0.8])
def test_1d_spectrum_approaches_plane_waves(k):
    """Continuum eigenvalues of -1/2 d^2 - i k d + k^2/2 on a periodic interval:
    1/2 (k + 2 pi m / L)^2; spectral elements resolve the low ones."""
    L, n_el, p = 6.0, 6, 7
    ev = np.linalg.eigvalsh(kpoint.operator_1d_periodic(L, n_el, p, k))
    m = np.arange(-4, 5)
    exact = np.sort(0.5 * (k + 2 * np.pi * m / L) ** 2)
    np.testing.assert_allclose(ev[:5], exact[:5], rtol=1e-8, atol=1e-10)


def test_k_zero_null_vector():
    L, n_el, p = 5.0, 2, 4
    n = n_el * p
    H = kpoint.htilde_k_csr(L, n_el, p, np.zeros(n ** 3), [0.0, 0.0, 0.0])
    _, _, M = kpoint.assemble_periodic(L, n_el, p)
    v = np.sqrt(M)
    assert np.abs(H @ v).max() < 1e-12 * np.abs(H).max()
    # the periodic 3D mass is the product of periodic 1D masses
    _, w = fem.gll(p)
    m1 = np.zeros(n)
    for e in range(n_el):
        m1[np.arange(e * p, e * p + p + 1) % n] += 0.5 * (L / n_el) * w
    np.testing.assert_allclose(M, np.kron(m1, np.kron(m1, m1)), rtol=1e-14)


def test_kronecker_apply_matches_csr_with_potential():
    L, n_el, p = 6.0, 2, 3
    k = np.array([0.2, 0.45, -0.3])
    xyz = kpoint.dof_coords_periodic(L, n_el, p)
    V = workload.eval_wells(workload.draw_wells(2, L, 8, (1.0, 2.0), (0.5, 1.0)), xyz)
    H = kpoint.htilde_k_csr(L, n_el, p, V, k)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((H.shape[0], 5)) + 1j * rng.standard_normal((H.shape[0], 5))
    A = [kpoint.operator_1d_periodic(L, n_el, p, kd) for kd in k]
    np.testing.assert_allclose(kpoint.apply_kron_k(*A, V, X), H @ X, rtol=0, atol=1e-12 * np.abs(H @ X).max())


def test_periodic_map_and_colouring():
    """Every periodic dof appears; within one colour no two cells share a dof
    (n_el even), and each dof has exactly one first-touch cell by the parity rule."""
    n_el, p = 4, 3
    cmap = kpoint.cell_dof_map_periodic(n_el, p)
    col = fem.cell_colors(n_el)
    nd = (n_el * p) ** 3
    assert set(np.unique(cmap)) == set(range(nd))
    for c in range(8):
        d = cmap[col == c].reshape(-1)
        assert d.size == np.unique(d).size
    q = p + 1
    first = np.zeros(nd, dtype=int)
    for e in range(cmap.shape[0]):
        ex, ey, ez = e % n_el, (e // n_el) % n_el, e // n_el ** 2
        for l in range(q ** 3):
            a, b, cc = l % q, (l // q) % q, l // q ** 2
            fx = (0 < a < q - 1) or ex % 2 == 0
            fy = (0 < b < q - 1) or ey % 2 == 0
            fz = (0 < cc < q - 1) or ez % 2 == 0
            first[cmap[e, l]] += fx and fy and fz
    assert np.all(first == 1)
