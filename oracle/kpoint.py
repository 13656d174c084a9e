"""Oracle: the periodic (Bloch) Kohn-Sham operator at a k-point, FP64 / complex128
on the CPU.  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2.1 eq. ksproblemPer: on the periodic cell Omega_p = [0, L]^3 the
Bloch-periodic part u of psi = e^{i k.x} u solves

    (-1/2 Laplacian - i k.grad + 1/2 |k|^2 + V) u = eps u,   u periodic.

Discretised with the same GLL spectral elements (Sec. 2.4) and periodic
numbering (node index I = (ex p + a) mod (n_el p), n = n_el p nodes per
direction, no Dirichlet nodes), the Galerkin matrix is

    H_k = K + 1/2 |k|^2 M + M V - i (k_x G_x + k_y G_y + k_z G_z),

K the stiffness of -1/2 Laplacian (``fem.cell_stiffness``), M the diagonal GLL
mass, and G_d[j, l] = int N_j d_d N_l.  With the GLL rule on the cell the first
derivative term is G_x^e[(a',b',c'), (a,b,c)] = (h/2)^2 w_a' w_b' w_c' D[a', a]
delta_b'b delta_c'c (and likewise in y, z); the integrand is of degree 2p - 1 in
the derivative direction, which the (p+1)-point GLL rule integrates exactly, so
after periodic assembly G is exactly antisymmetric and H_k is Hermitian.
Standard form Htilde_k = M^-1/2 H_k M^-1/2 (eq. hep).

* ``cell_dof_map_periodic``, ``cell_convection``, ``assemble_periodic``,
  ``htilde_k_csr``           -- the operator above, assembled cell by cell;
* ``operator_1d_periodic``   -- the 1D factor m^-1/2 (1/2 K1D - i k C1D +
  1/2 k^2 m) m^-1/2 on n periodic nodes;
* ``apply_kron_k``           -- Htilde_k X = (A_x (+) A_y (+) A_z) X + V X, the
  Kronecker-sum form (serves the full-size meshes);
* ``dof_coords_periodic``.

Pins (tests/test_oracle_kpoint.py): G antisymmetric after assembly;
the cell G against Gauss-Legendre quadrature of the general Lagrange basis
(exactness); Htilde_k Hermitian; the assembled operator against the
Kronecker sum of 1D operators; the 1D spectrum against the continuum plane-wave
values 1/2 (k + 2 pi m / L)^2; k = 0: the null vector M^1/2 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem


def cell_dof_map_periodic(n_el: int, p: int) -> np.ndarray:
    """int32 [n_cells, (p+1)^3]: dof = I + n J + n^2 K, I = (ex p + a) mod n."""
    n = n_el * p
    q = p + 1
    out = np.empty((n_el ** 3, q ** 3), dtype=np.int32)
    for ez in range(n_el):
        for ey in range(n_el):
            for ex in range(n_el):
                e = ex + n_el * ey + n_el * n_el * ez
                for c in range(q):
                    for b in range(q):
                        for a in range(q):
                            I, J, K = (ex * p + a) % n, (ey * p + b) % n, (ez * p + c) % n
                            out[e, a + q * b + q * q * c] = I + n * J + n * n * K
    return out


def dof_coords_periodic(L: float, n_el: int, p: int) -> np.ndarray:
    """[n^3, 3] node coordinates in dof order (I = 0 .. n - 1 at x = 0 .. < L)."""
    x = fem.node_coords_1d(L, n_el, p)[:-1]
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)


def cell_convection(p: int, h: float):
    """(G_x, G_y, G_z) cell matrices [n_loc, n_loc] of int N_j d_d N_l by the GLL
    rule, local node l = a + (p+1) b + (p+1)^2 c."""
    _, w = fem.gll(p)
    D = fem.deriv_matrix(p)                     # D[q, a] = l_a'(xi_q)
    W = np.diag(w)
    C1 = W @ D                                  # [a', a] = w_a' l_a'(xi_a')
    s = (h / 2.0) ** 2
    gx = s * np.kron(W, np.kron(W, C1))
    gy = s * np.kron(W, np.kron(C1, W))
    gz = s * np.kron(C1, np.kron(W, W))
    return gx, gy, gz


def assemble_periodic(L: float, n_el: int, p: int):
    """(K, (G_x, G_y, G_z), M): CSR stiffness of -1/2 Laplacian, CSR first-derivative
    matrices and the diagonal mass, assembled with periodic numbering."""
    h = L / n_el
    Ke = fem.cell_stiffness(p, h)
    Me = fem.cell_mass(p, h)
    Ge = cell_convection(p, h)
    cmap = cell_dof_map_periodic(n_el, p)
    nd = (n_el * p) ** 3
    rows = np.repeat(cmap, cmap.shape[1], axis=1).reshape(-1)
    cols = np.tile(cmap, (1, cmap.shape[1])).reshape(-1)
    nc = cmap.shape[0]

    def build(Ae):
        vals = np.tile(Ae.reshape(-1), nc)
        A = sp.coo_matrix((vals, (rows, cols)), shape=(nd, nd)).tocsr()
        A.sum_duplicates()
        return A

    M = np.zeros(nd)
    np.add.at(M, cmap.reshape(-1), np.tile(Me, nc))
    return build(Ke), tuple(build(g) for g in Ge), M


def htilde_k_csr(L: float, n_el: int, p: int, V: np.ndarray, k) -> sp.csr_matrix:
    """Htilde_k = M^-1/2 (K - i k.G) M^-1/2 + diag(V + |k|^2 / 2), complex CSR."""
    K, G, M = assemble_periodic(L, n_el, p)
    k = np.asarray(k, dtype=np.float64)
    s = sp.diags(1.0 / np.sqrt(M))
    H = s @ (K.astype(np.complex128) - 1j * (k[0] * G[0] + k[1] * G[1] + k[2] * G[2])) @ s
    return (H + sp.diags(np.asarray(V, dtype=np.float64) + 0.5 * float(k @ k))).tocsr()


def operator_1d_periodic(L: float, n_el: int, p: int, k: float) -> np.ndarray:
    """m^-1/2 (1/2 K1D - i k C1D + 1/2 k^2 m) m^-1/2 on the n = n_el p periodic 1D
    nodes (C1D[j, l] = int phi_j phi_l')."""
    h = L / n_el
    _, w = fem.gll(p)
    K1 = fem.stiffness_1d_ref(p)
    D = fem.deriv_matrix(p)
    C1 = np.diag(w) @ D
    n = n_el * p
    K1D = np.zeros((n, n))
    C1D = np.zeros((n, n))
    m = np.zeros(n)
    for e in range(n_el):
        idx = np.arange(e * p, e * p + p + 1) % n
        K1D[np.ix_(idx, idx)] += (2.0 / h) * K1
        C1D[np.ix_(idx, idx)] += C1
        m[idx] += (h / 2.0) * w
    d = 1.0 / np.sqrt(m)
    return d[:, None] * (0.5 * K1D - 1j * k * C1D + 0.5 * k * k * np.diag(m)) * d[None, :]


def apply_kron_k(Ax: np.ndarray, Ay: np.ndarray, Az: np.ndarray, V: np.ndarray, X: np.ndarray) -> np.ndarray:
    """(A_x (+) A_y (+) A_z + diag(V)) X, dof = I + n J + n^2 K, complex X [n^3, c]."""
    n = Ax.shape[0]
    X = np.asarray(X, dtype=np.complex128)
    one = X.ndim == 1
    Xc = X.reshape(n ** 3, -1)
    c = Xc.shape[1]
    Xr = Xc.reshape(n, n, n, c)                                      # [K, J, I, col]
    Y = np.matmul(Ax, Xr.reshape(n * n, n, c)).reshape(n, n, n, c)  # along I
    Y += np.matmul(Ay, Xr.reshape(n, n, n * c)).reshape(n, n, n, c)  # along J
    Y += (Az @ Xr.reshape(n, n * n * c)).reshape(n, n, n, c)        # along K
    Y = Y.reshape(n ** 3, c) + np.asarray(V, dtype=np.float64)[:, None] * Xc
    return Y.reshape(-1) if one else Y


__all__ = ["cell_dof_map_periodic", "dof_coords_periodic", "cell_convection", "assemble_periodic",
           "htilde_k_csr", "operator_1d_periodic", "apply_kron_k"]
