"""Oracle: spectral (GLL) finite-element discretisation of H = -1/2 Laplacian + V.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain FP64 numpy/scipy.

Follows the paper's Sec. 2.4 (discrete Kohn-Sham equations):

* C0 Lagrange basis interpolating at Gauss-Lobatto-Legendre (GLL) nodes (eq. fem);
* local Hamiltonian  H_jk = 1/2 int grad N_j . grad N_k + int V N_j N_k  (eq. discreteHam);
* mass matrix        M_jk = int N_j N_k, made diagonal by GLL quadrature;
* standard form      Htilde = M^-1/2 H M^-1/2  (eq. hep), eigenvectors psi_hat = M^-1/2 psi_tilde.

Readings where the paper is silent:

* all three integrals use the (p+1)^3-point GLL rule collocated with the nodes,
  so the potential term is diag(M_j V(x_j)) and Htilde = M^-1/2 K M^-1/2 + diag(V);
* the domain is [0,L]^3 with homogeneous Dirichlet conditions: boundary nodes
  carry no degree of freedom;
* numbering: interior node (I,J,K), 1 <= I,J,K <= n with n = n_el p - 1, has
  dof = (I-1) + n (J-1) + n^2 (K-1); cell e = ex + n_el ey + n_el^2 ez; local
  node l = a + (p+1) b + (p+1)^2 c with I = ex p + a; map entry -1 marks a
  Dirichlet node; cell colour = (ex&1) + 2 (ey&1) + 4 (ez&1).

Pins (tests/test_oracle_fem.py): GLL rule against the library roots of P'_p and
polynomial exactness; D against derivatives of monomials; cell stiffness
symmetric, PSD with the constants as its only kernel; map bijection,
multiplicities and colouring; CSR assembly against the Kronecker-sum form and
against a brute-force quadrature assembly written with general Lagrange
evaluation; V=0 spectrum against sums of 1D eigenvalues and against the
continuum particle-in-a-box values; the harmonic oscillator limit.  The
Kronecker-product diagonal mass (``mass_diag_kron``) against the assembled M
(tests/test_oracle_density.py); the 1D reference stiffness against closed forms
and exact polynomial integrals; the 1D mass against its closed forms.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------
# GLL rule and Lagrange basis on [-1, 1]
# --------------------------------------------------------------------------

def legendre(p: int, x):
    """(P_p(x), P_p'(x)) by the three-term (Bonnet) recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0, p1 = np.ones_like(x), x.copy()
    d0, d1 = np.zeros_like(x), np.ones_like(x)
    if p == 0:
        return p0, d0
    for k in range(1, p):
        p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
        d2 = d0 + (2 * k + 1) * p1          # P'_{k+1} = P'_{k-1} + (2k+1) P_k
        p0, p1, d0, d1 = p1, p2, d1, d2
    return p1, d1


def gll(p: int):
    """GLL nodes (ascending, endpoints +-1 and the roots of P'_p) and weights
    w_a = 2 / (p (p+1) P_p(xi_a)^2).  Interior roots by Newton's method on P'_p,
    with P''_p from Legendre's equation (1-x^2) P'' = 2x P' - p(p+1) P."""
    assert p >= 1
    x = -np.cos(np.pi * np.arange(p + 1) / p)   # Chebyshev-Lobatto start
    for _ in range(100):
        P, dP = legendre(p, x[1:-1])
        d2P = (2.0 * x[1:-1] * dP - p * (p + 1) * P) / (1.0 - x[1:-1] ** 2)
        step = dP / d2P
        x[1:-1] -= step
        if np.max(np.abs(step), initial=0.0) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    P, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P ** 2)
    return x, w


def lagrange_eval(nodes: np.ndarray, x) -> np.ndarray:
    """Values L[i, a] = l_a(x_i) of the Lagrange basis on ``nodes`` (product formula)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.shape[0]
    out = np.ones((x.shape[0], n))
    for a in range(n):
        for k in range(n):
            if k != a:
                out[:, a] *= (x - nodes[k]) / (nodes[a] - nodes[k])
    return out


def lagrange_deriv_eval(nodes: np.ndarray, x) -> np.ndarray:
    """Derivatives L'[i, a] = l_a'(x_i): the product rule applied to the product formula."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.shape[0]
    out = np.zeros((x.shape[0], n))
    for a in range(n):
        for m in range(n):
            if m == a:
                continue
            term = np.full(x.shape[0], 1.0 / (nodes[a] - nodes[m]))
            for k in range(n):
                if k != a and k != m:
                    term *= (x - nodes[k]) / (nodes[a] - nodes[k])
            out[:, a] += term
    return out


def deriv_matrix(p: int) -> np.ndarray:
    """D[q, a] = l_a'(xi_q) at the GLL nodes."""
    xi, _ = gll(p)
    return lagrange_deriv_eval(xi, xi)


# --------------------------------------------------------------------------
# Reference cell matrices
# --------------------------------------------------------------------------

def stiffness_1d_ref(p: int) -> np.ndarray:
    """K1[a, a'] = sum_q w_q D[q,a] D[q,a'] = int_{-1}^{1} l_a' l_a'' (exact: degree 2p-2)."""
    _, w = gll(p)
    D = deriv_matrix(p)
    return D.T @ (w[:, None] * D)


def cell_stiffness(p: int, h: float) -> np.ndarray:
    """Cell matrix of 1/2 int grad N . grad N on a cube of side h, GLL quadrature:
    1/2 (h/2) [K1 (x) W (x) W + W (x) K1 (x) W + W (x) W (x) K1] with W = diag(w),
    local node l = a + (p+1) b + (p+1)^2 c (x fastest)."""
    _, w = gll(p)
    K1 = stiffness_1d_ref(p)
    W = np.diag(w)
    kx = np.kron(W, np.kron(W, K1))
    ky = np.kron(W, np.kron(K1, W))
    kz = np.kron(K1, np.kron(W, W))
    return 0.5 * (h / 2.0) * (kx + ky + kz)


def cell_mass(p: int, h: float) -> np.ndarray:
    """Diagonal of the GLL-quadrature cell mass matrix: (h/2)^3 w_a w_b w_c."""
    _, w = gll(p)
    return (h / 2.0) ** 3 * np.kron(w, np.kron(w, w))


# --------------------------------------------------------------------------
# Mesh numbering, maps and colouring
# --------------------------------------------------------------------------

def sizes(n_el: int, p: int):
    """n interior nodes per direction, n_dof = n^3, cells and local nodes."""
    n = n_el * p - 1
    return dict(n=n, n_dof=n ** 3, n_cells=n_el ** 3, n_loc=(p + 1) ** 3)


def cell_dof_map(n_el: int, p: int) -> np.ndarray:
    """int32 [n_cells, (p+1)^3]; -1 marks a node on the Dirichlet boundary."""
    n = n_el * p - 1
    q = p + 1
    out = np.empty((n_el ** 3, q ** 3), dtype=np.int32)
    for ez in range(n_el):
        for ey in range(n_el):
            for ex in range(n_el):
                e = ex + n_el * ey + n_el * n_el * ez
                for c in range(q):
                    for b in range(q):
                        for a in range(q):
                            I, J, K = ex * p + a, ey * p + b, ez * p + c
                            l = a + q * b + q * q * c
                            if min(I, J, K) == 0 or max(I, J, K) == n_el * p:
                                out[e, l] = -1
                            else:
                                out[e, l] = (I - 1) + n * (J - 1) + n * n * (K - 1)
    return out


def cell_colors(n_el: int) -> np.ndarray:
    """uint8 [n_cells]: (ex&1) + 2 (ey&1) + 4 (ez&1)."""
    out = np.empty(n_el ** 3, dtype=np.uint8)
    for ez in range(n_el):
        for ey in range(n_el):
            for ex in range(n_el):
                out[ex + n_el * ey + n_el * n_el * ez] = (ex & 1) + 2 * (ey & 1) + 4 * (ez & 1)
    return out


def node_coords_1d(L: float, n_el: int, p: int) -> np.ndarray:
    """x of all 1D nodes I = 0 .. n_el p (boundary included)."""
    xi, _ = gll(p)
    h = L / n_el
    x = np.empty(n_el * p + 1)
    for ex in range(n_el):
        for a in range(p + 1):
            x[ex * p + a] = ex * h + (1.0 + xi[a]) * h / 2.0
    x[0], x[-1] = 0.0, L
    return x


def dof_coords(L: float, n_el: int, p: int) -> np.ndarray:
    """[n_dof, 3] coordinates of the interior nodes in dof order."""
    x = node_coords_1d(L, n_el, p)[1:-1]
    n = x.shape[0]
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")   # index [K, J, I], I fastest in dof
    return np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)


# --------------------------------------------------------------------------
# Assembled operators
# --------------------------------------------------------------------------

def assemble(L: float, n_el: int, p: int):
    """Global stiffness K (CSR, interior DoFs) and diagonal mass M by summing the
    cell matrices through the cell map, dropping Dirichlet nodes."""
    h = L / n_el
    Ke = cell_stiffness(p, h)
    Me = cell_mass(p, h)
    cmap = cell_dof_map(n_el, p)
    nd = (n_el * p - 1) ** 3
    rows, cols, vals = [], [], []
    M = np.zeros(nd)
    for e in range(cmap.shape[0]):
        g = cmap[e]
        live = np.nonzero(g >= 0)[0]
        gi = g[live]
        rows.append(np.repeat(gi, live.size))
        cols.append(np.tile(gi, live.size))
        vals.append(Ke[np.ix_(live, live)].reshape(-1))
        np.add.at(M, gi, Me[live])
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nd, nd)).tocsr()
    K.sum_duplicates()
    return K, M


def mass_1d(L: float, n_el: int, p: int) -> np.ndarray:
    """Diagonal 1D GLL mass on the n_el p - 1 interior nodes: sum over the 1D
    elements of (h/2) w_a at each element's nodes."""
    h = L / n_el
    _, w = gll(p)
    m = np.zeros(n_el * p + 1)
    for e in range(n_el):
        m[e * p:e * p + p + 1] += 0.5 * h * w
    return m[1:-1]


def mass_diag_kron(L: float, n_el: int, p: int) -> np.ndarray:
    """The 3D diagonal GLL mass as the product m(I) m(J) m(K) of 1D masses
    (the tensor-product rule), dof = I + n J + n^2 K; no assembly loop, so it
    serves the full-size meshes."""
    m = mass_1d(L, n_el, p)
    return np.kron(m, np.kron(m, m))


def htilde_csr(L: float, n_el: int, p: int, V: np.ndarray):
    """Htilde = M^-1/2 (K + diag(M V)) M^-1/2 = M^-1/2 K M^-1/2 + diag(V), CSR."""
    K, M = assemble(L, n_el, p)
    s = sp.diags(1.0 / np.sqrt(M))
    return (s @ K @ s + sp.diags(np.asarray(V, dtype=np.float64))).tocsr()


def operator_1d(L: float, n_el: int, p: int) -> np.ndarray:
    """A = 1/2 M1^-1/2 K1D M1^-1/2 on the n = n_el p - 1 interior 1D nodes, with
    K1D = sum_e (2/h) K1 and M1 = sum_e (h/2) w assembled over 1D elements."""
    h = L / n_el
    _, w = gll(p)
    K1 = stiffness_1d_ref(p)
    n1 = n_el * p + 1
    K1D = np.zeros((n1, n1))
    M1 = np.zeros(n1)
    for e in range(n_el):
        s = slice(e * p, e * p + p + 1)
        K1D[s, s] += (2.0 / h) * K1
        M1[s] += (h / 2.0) * w
    K1D, M1 = K1D[1:-1, 1:-1], M1[1:-1]
    d = 1.0 / np.sqrt(M1)
    return 0.5 * d[:, None] * K1D * d[None, :]


def apply_kron(A: np.ndarray, V: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Htilde X with Htilde = A(+)A(+)A + diag(V) (Kronecker sum, dof = I + nJ + n^2 K)."""
    n = A.shape[0]
    X = np.asarray(X, dtype=np.float64)
    one = X.ndim == 1
    Xc = X.reshape(n ** 3, -1)
    c = Xc.shape[1]
    Xr = Xc.reshape(n, n, n, c)                                   # [K, J, I, col]
    Y = np.matmul(A, Xr.reshape(n * n, n, c))                     # along I
    Y = Y.reshape(n, n, n, c)
    Y += np.matmul(A, Xr.reshape(n, n, n * c)).reshape(n, n, n, c)   # along J
    Y += (A @ Xr.reshape(n, n * n * c)).reshape(n, n, n, c)       # along K
    Y = Y.reshape(n ** 3, c) + np.asarray(V, dtype=np.float64)[:, None] * Xc
    return Y.reshape(-1) if one else Y


def upper_bound(A: np.ndarray, V: np.ndarray) -> float:
    """b >= lambda_max(Htilde): 3 lambda_max(A) + max V (Weyl, for the Kronecker sum plus a diagonal)."""
    return 3.0 * float(np.linalg.eigvalsh(A)[-1]) + float(np.max(V))


def brute_force_htilde(L: float, n_el: int, p: int, vfun) -> np.ndarray:
    """Dense Htilde by direct GLL quadrature of the basis functions on every cell
    (general Lagrange evaluation, no tensor shortcuts).  For tiny meshes only."""
    xi, w = gll(p)
    q = p + 1
    h = L / n_el
    Lv = lagrange_eval(xi, xi)          # [quad, a]
    Ld = lagrange_deriv_eval(xi, xi)    # [quad, a]
    cmap = cell_dof_map(n_el, p)
    nd = (n_el * p - 1) ** 3
    H = np.zeros((nd, nd))
    Mf = np.zeros((nd, nd))
    jac = (h / 2.0) ** 3
    for ez in range(n_el):
        for ey in range(n_el):
            for ex in range(n_el):
                e = ex + n_el * ey + n_el * n_el * ez
                g = cmap[e]
                for qz in range(q):
                    for qy in range(q):
                        for qx in range(q):
                            wq = w[qx] * w[qy] * w[qz] * jac
                            xq = np.array([ex * h + (1 + xi[qx]) * h / 2,
                                           ey * h + (1 + xi[qy]) * h / 2,
                                           ez * h + (1 + xi[qz]) * h / 2])
                            vq = vfun(xq[None, :])[0]
                            Nv = np.zeros(q ** 3)
                            G = np.zeros((q ** 3, 3))
                            for c in range(q):
                                for b in range(q):
                                    for a in range(q):
                                        l = a + q * b + q * q * c
                                        Nv[l] = Lv[qx, a] * Lv[qy, b] * Lv[qz, c]
                                        G[l, 0] = (2 / h) * Ld[qx, a] * Lv[qy, b] * Lv[qz, c]
                                        G[l, 1] = (2 / h) * Lv[qx, a] * Ld[qy, b] * Lv[qz, c]
                                        G[l, 2] = (2 / h) * Lv[qx, a] * Lv[qy, b] * Ld[qz, c]
                            live = np.nonzero(g >= 0)[0]
                            gi = g[live]
                            H[np.ix_(gi, gi)] += wq * (0.5 * G[live] @ G[live].T
                                                       + vq * np.outer(Nv[live], Nv[live]))
                            Mf[np.ix_(gi, gi)] += wq * np.outer(Nv[live], Nv[live])
    m = np.diag(Mf).copy()
    s = 1.0 / np.sqrt(m)
    return s[:, None] * H * s[None, :], Mf


__all__ = ["legendre", "gll", "lagrange_eval", "lagrange_deriv_eval", "deriv_matrix",
           "stiffness_1d_ref", "cell_stiffness", "cell_mass", "sizes", "cell_dof_map",
           "cell_colors", "node_coords_1d", "dof_coords", "assemble", "htilde_csr",
           "operator_1d", "apply_kron", "upper_bound", "brute_force_htilde"]
