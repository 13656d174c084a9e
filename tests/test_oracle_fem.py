"""Pins of the oracle's finite-element discretisation (CPU only).

Each test checks the oracle against something other than itself: closed
forms, library routines, invariants, or a brute-force assembly that shares
none of the tensor-product shortcuts.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import fem
import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _eval(expr: str) -> float:
    return float(eval(expr, {"sqrt": math.sqrt, "__builtins__": {}}))


# ---------------------------------------------------------------- GLL rule

@pytest.mark.parametrize("p", list(range(1, 13)))
def test_gll_nodes_match_library_roots(p):
    xi, w = fem.gll(p)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    if p >= 2:
        roots = np.sort(np.polynomial.legendre.Legendre.basis(p).deriv().roots().real)
        np.testing.assert_allclose(xi[1:-1], roots, rtol=0, atol=1e-14)
    np.testing.assert_allclose(xi, -xi[::-1], atol=1e-15)
    np.testing.assert_allclose(w, w[::-1], atol=1e-15)
    assert abs(w.sum() - 2.0) < 1e-14


@pytest.mark.parametrize("p", list(range(1, 13)))
def test_gll_polynomial_exactness(p):
    xi, w = fem.gll(p)
    for k in range(0, 2 * p):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14, k
    # degree 2p is not integrated exactly (the rule is Lobatto, not Gauss)
    exact = 2.0 / (2 * p + 1)
    assert abs(np.dot(w, xi ** (2 * p)) - exact) > 1e-9


def test_gll_closed_forms():
    with open(os.path.join(GOLDEN, "gll_closed_form.json")) as f:
        g = json.load(f)
    for p, rule in g["rules"].items():
        xi, w = fem.gll(int(p))
        np.testing.assert_allclose(xi, [_eval(s) for s in rule["nodes"]], atol=1e-15)
        np.testing.assert_allclose(w, [_eval(s) for s in rule["weights"]], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_derivative_matrix_on_monomials(p):
    xi, _ = fem.gll(p)
    D = fem.deriv_matrix(p)
    for k in range(0, p + 1):
        f = xi ** k
        df = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        np.testing.assert_allclose(D @ f, df, atol=1e-12 * max(1, k * k))
    # standard corner identity and zero interior diagonal
    assert abs(D[0, 0] + p * (p + 1) / 4.0) < 1e-11
    assert abs(D[p, p] - p * (p + 1) / 4.0) < 1e-11
    if p >= 2:
        assert np.max(np.abs(np.diag(D)[1:-1])) < 1e-11


# ---------------------------------------------------------------- cell matrices

@pytest.mark.parametrize("p", [2, 4, 5, 6, 7])
def test_cell_stiffness_invariants(p):
    h = 1.7
    K = fem.cell_stiffness(p, h)
    assert np.max(np.abs(K - K.T)) < 1e-14 * np.max(np.abs(K))
    assert np.max(np.abs(K @ np.ones(K.shape[0]))) < 1e-13 * np.max(np.abs(K))
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-12 * ev[-1]
    assert ev[1] > 1e-6 * ev[-1]          # one-dimensional kernel (the constants)


@pytest.mark.parametrize("p", [2, 3, 4, 6])
def test_cell_stiffness_energy_of_quadratic(p):
    """u = x^2 on [0,h]^3: 1/2 int |grad u|^2 = 1/2 int 4x^2 = (2/3) h^5 exactly
    (integrand degree 2 in x, constant in y, z: every GLL rule p >= 2 is exact)."""
    h = 1.3
    xi, _ = fem.gll(p)
    x = (1 + xi) * h / 2
    q = p + 1
    u = np.tile(x ** 2, q * q)            # l = a + q b + q^2 c, depends on a only
    K = fem.cell_stiffness(p, h)
    assert abs(u @ K @ u - (2.0 / 3.0) * h ** 5) < 1e-12 * h ** 5
    # a function of z only exercises the z term of the tensor sum
    uz = np.repeat(x ** 2, q * q)
    assert abs(uz @ K @ uz - (2.0 / 3.0) * h ** 5) < 1e-12 * h ** 5


def test_stiffness_1d_closed_forms():
    """int l_a' l_b' on [-1, 1] for linear and quadratic Lagrange elements."""
    np.testing.assert_allclose(fem.stiffness_1d_ref(1), [[0.5, -0.5], [-0.5, 0.5]], rtol=0, atol=1e-15)
    k2 = np.array([[7.0, -8.0, 1.0], [-8.0, 16.0, -8.0], [1.0, -8.0, 7.0]]) / 6.0
    np.testing.assert_allclose(fem.stiffness_1d_ref(2), k2, rtol=0, atol=1e-14)


@pytest.mark.parametrize("p", [3, 5, 7, 9])
def test_stiffness_1d_against_exact_polynomial_integrals(p):
    """Each Lagrange basis polynomial built from its roots (the other nodes),
    differentiated and the products integrated exactly as polynomials: no
    quadrature and no derivative matrix involved."""
    from numpy.polynomial import polynomial as Pn
    x, _ = fem.gll(p)
    dl = []
    for a in range(p + 1):
        c = Pn.polyfromroots(np.delete(x, a))
        dl.append(Pn.polyder(c / Pn.polyval(x[a], c)))
    K = np.empty((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            prim = Pn.polyint(Pn.polymul(dl[i], dl[j]))
            K[i, j] = Pn.polyval(1.0, prim) - Pn.polyval(-1.0, prim)
    np.testing.assert_allclose(fem.stiffness_1d_ref(p), K, rtol=0, atol=1e-11 * np.abs(K).max())


def test_cell_mass_volume():
    for p in [2, 4, 7]:
        h = 2.5
        assert abs(fem.cell_mass(p, h).sum() - h ** 3) < 1e-13 * h ** 3


@pytest.mark.parametrize("L,n_el,p", [(6.0, 1, 4), (9.0, 3, 4), (10.0, 4, 5), (7.5, 5, 2)])
def test_mass_1d_closed_forms(L, n_el, p):
    """The 1D GLL mass integrates constants exactly: the interior nodal masses
    add up to L less the two wall nodes' (h/2) w_0 = h / (p (p + 1)) each;
    a node on an element boundary carries twice the end weight, and the
    pattern repeats with period p."""
    m = fem.mass_1d(L, n_el, p)
    h = L / n_el
    assert m.shape == (n_el * p - 1,)
    w_end = h / (p * (p + 1))
    assert abs(m.sum() - (L - 2 * w_end)) < 1e-13 * L
    shared = np.arange(1, n_el * p)[np.arange(1, n_el * p) % p == 0] - 1
    np.testing.assert_allclose(m[shared], 2 * w_end, rtol=1e-14)
    if n_el > 1:
        np.testing.assert_allclose(m[p:], m[:-p], rtol=1e-14)


@pytest.mark.parametrize("n_el,p", [(1, 2), (2, 3), (3, 5)])
def test_sizes_agree_with_the_map(n_el, p):
    s = fem.sizes(n_el, p)
    cmap = fem.cell_dof_map(n_el, p)
    assert cmap.shape == (s["n_cells"], s["n_loc"])
    assert int(cmap.max()) + 1 == s["n_dof"] == s["n"] ** 3
    assert fem.dof_coords(1.0, n_el, p).shape == (s["n_dof"], 3)


# ---------------------------------------------------------------- numbering

@pytest.mark.parametrize("n_el,p", [(1, 2), (2, 3), (4, 4), (3, 5), (4, 2)])
def test_map_bijection_and_multiplicity(n_el, p):
    cmap = fem.cell_dof_map(n_el, p)
    n = n_el * p - 1
    nd = n ** 3
    live = cmap[cmap >= 0]
    counts = np.bincount(live, minlength=nd)
    assert counts.shape[0] == nd and counts.min() >= 1
    assert set(np.unique(counts)).issubset({1, 2, 4, 8})
    # combinatorics: a node shared along k axes (element-boundary coordinate) lies in 2^k cells
    I = np.arange(1, n + 1)
    shared = (I % p == 0).astype(int)
    expect = (2 ** (shared[None, None, :] + shared[None, :, None] + shared[:, None, None])).reshape(-1)
    np.testing.assert_array_equal(counts, expect)
    # every interior node appears exactly once per containing cell
    for e in range(cmap.shape[0]):
        g = cmap[e][cmap[e] >= 0]
        assert np.unique(g).size == g.size


@pytest.mark.parametrize("n_el,p", [(2, 3), (4, 4), (6, 2)])
def test_colouring(n_el, p):
    cmap = fem.cell_dof_map(n_el, p)
    col = fem.cell_colors(n_el)
    for c in range(8):
        cells = np.nonzero(col == c)[0]
        assert cells.size == n_el ** 3 // 8
        g = cmap[cells]
        g = g[g >= 0]
        assert np.unique(g).size == g.size      # same-colour cells share no DoF


def test_dof_coords_follow_the_map():
    L, n_el, p = 7.0, 3, 3
    xyz = fem.dof_coords(L, n_el, p)
    xi, _ = fem.gll(p)
    h = L / n_el
    cmap = fem.cell_dof_map(n_el, p)
    q = p + 1
    for e in [0, 5, 13, 26]:
        ex, ey, ez = e % n_el, (e // n_el) % n_el, e // (n_el * n_el)
        for l in range(q ** 3):
            d = cmap[e, l]
            if d < 0:
                continue
            a, b, c = l % q, (l // q) % q, l // (q * q)
            want = [ex * h + (1 + xi[a]) * h / 2, ey * h + (1 + xi[b]) * h / 2, ez * h + (1 + xi[c]) * h / 2]
            np.testing.assert_allclose(xyz[d], want, atol=1e-13)


# ---------------------------------------------------------------- assembled operator

@pytest.mark.parametrize("n_el,p", [(2, 2), (3, 4), (4, 4), (2, 6)])
def test_csr_equals_kronecker_sum(n_el, p):
    L = 10.0
    nd = (n_el * p - 1) ** 3
    rng = np.random.default_rng(n_el * 10 + p)
    V = rng.uniform(-3, 1, nd)
    H = fem.htilde_csr(L, n_el, p, V)
    assert abs(H - H.T).max() < 1e-13 * abs(H).max()
    A = fem.operator_1d(L, n_el, p)
    X = rng.standard_normal((nd, 7))
    Y1 = H @ X
    Y2 = fem.apply_kron(A, V, X)
    assert np.max(np.abs(Y1 - Y2)) < 1e-14 * np.max(np.abs(Y1)) * 10


@pytest.mark.parametrize("n_el,p", [(1, 2), (1, 3), (1, 4), (2, 2), (2, 3), (2, 4)])
def test_brute_force_quadrature_assembly(n_el, p):
    L = 6.0
    vfun = lambda x: np.sin(x[:, 0]) + 0.1 * x[:, 1] - 0.3 * np.cos(x[:, 2])
    Hb, Mf = fem.brute_force_htilde(L, n_el, p, vfun)
    # GLL quadrature makes the mass matrix diagonal (Sec. 2.4)
    assert np.max(np.abs(Mf - np.diag(np.diag(Mf)))) == 0.0
    V = vfun(fem.dof_coords(L, n_el, p))
    Hc = fem.htilde_csr(L, n_el, p, V).toarray()
    assert np.max(np.abs(Hb - Hc)) < 1e-13 * max(1.0, np.max(np.abs(Hb)))


# ---------------------------------------------------------------- spectra

@pytest.mark.parametrize("n_el,p", [(2, 3), (3, 3), (2, 5)])
def test_v0_spectrum_is_sum_of_1d_spectra(n_el, p):
    L = 8.0
    nd = (n_el * p - 1) ** 3
    H = fem.htilde_csr(L, n_el, p, np.zeros(nd)).toarray()
    ev = np.linalg.eigvalsh(H)
    a = np.linalg.eigvalsh(fem.operator_1d(L, n_el, p))
    sums = np.sort((a[:, None, None] + a[None, :, None] + a[None, None, :]).reshape(-1))
    np.testing.assert_allclose(ev, sums, rtol=1e-13, atol=1e-13 * sums[-1])


@pytest.mark.parametrize("p", [3, 4])
def test_v0_convergence_order_2p(p):
    """Lowest 1D Dirichlet mode on [0, pi] is k^2/2 with k=1: error O(h^{2p})."""
    L = np.pi
    errs, hs = [], []
    for n_el in [2, 3, 4, 6]:
        a = np.linalg.eigvalsh(fem.operator_1d(L, n_el, p))
        errs.append(abs(a[0] - 0.5) / 0.5)
        hs.append(L / n_el)
    for i in range(3):
        order = math.log(errs[i] / errs[i + 1]) / math.log(hs[i] / hs[i + 1])
        assert abs(order - 2 * p) < 0.5, (i, order)


def test_box_ground_state_small_workload():
    """Particle in a box: lowest 3D level 3 pi^2 / (2 L^2) with its degeneracy pattern."""
    prob = workload.PROBLEMS["small"]
    a = np.linalg.eigvalsh(fem.operator_1d(prob.L, prob.n_el, prob.p))
    ev = np.sort((a[:, None, None] + a[None, :, None] + a[None, None, :]).reshape(-1))[:10]
    cont = np.sort([(i * i + j * j + k * k) * np.pi ** 2 / (2 * prob.L ** 2)
                    for i in range(1, 5) for j in range(1, 5) for k in range(1, 5)])[:10]
    # discretisation error grows with the mode number (~ (k h)^{2p}): ground state
    # to 1e-8, the first ten levels (k <= 3) to 2e-5; always from below here
    assert abs(ev[0] - cont[0]) < 1e-8 * cont[0]
    np.testing.assert_allclose(ev, cont, rtol=2e-5)
    assert np.all(ev <= cont + 1e-12)


def test_harmonic_oscillator_limit():
    """V = 1/2 w^2 |x - c|^2 is separable: 1D levels w (k + 1/2); the 3D spectrum
    w (n + 3/2) with degeneracy (n+1)(n+2)/2 (box error ~ exp(-w L^2/4) negligible)."""
    L, n_el, p, om = 14.0, 10, 7, 1.0
    A = fem.operator_1d(L, n_el, p)
    x = fem.node_coords_1d(L, n_el, p)[1:-1]
    a = np.linalg.eigvalsh(A + np.diag(0.5 * om ** 2 * (x - L / 2) ** 2))
    np.testing.assert_allclose(a[:6], om * (np.arange(6) + 0.5), rtol=1e-6)
    ev = np.sort((a[:, None, None] + a[None, :, None] + a[None, None, :]).reshape(-1))[:20]
    want = np.concatenate([np.full((n + 1) * (n + 2) // 2, om * (n + 1.5)) for n in range(4)])
    np.testing.assert_allclose(ev, want, rtol=1e-6)


def test_harmonic_3d_operator_is_separable():
    L, n_el, p, om = 8.0, 2, 4, 0.8
    xyz = fem.dof_coords(L, n_el, p)
    V = workload.harmonic(xyz, om, [L / 2] * 3)
    H = fem.htilde_csr(L, n_el, p, V).toarray()
    ev = np.linalg.eigvalsh(H)
    x = fem.node_coords_1d(L, n_el, p)[1:-1]
    a = np.linalg.eigvalsh(fem.operator_1d(L, n_el, p) + np.diag(0.5 * om ** 2 * (x - L / 2) ** 2))
    sums = np.sort((a[:, None, None] + a[None, :, None] + a[None, None, :]).reshape(-1))
    np.testing.assert_allclose(ev, sums, rtol=1e-12, atol=1e-12 * sums[-1])


def test_upper_bound_is_rigorous_and_tight():
    prob = workload.PROBLEMS["small"]
    xyz = fem.dof_coords(prob.L, prob.n_el, prob.p)
    V = workload.eval_wells(workload.problem_wells(prob), xyz)
    H = fem.htilde_csr(prob.L, prob.n_el, prob.p, V).toarray()
    lmax = np.linalg.eigvalsh(H)[-1]
    b = fem.upper_bound(fem.operator_1d(prob.L, prob.n_el, prob.p), V)
    assert b >= lmax and b - lmax < 0.02 * lmax
