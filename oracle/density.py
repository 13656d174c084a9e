"""Oracle: spectrum-splitting Rayleigh-Ritz and the electron density, FP64 on
the CPU.  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``fermi_dirac``          -- the orbital occupancy of Sec. 2.1:
  f(eps, mu) = 1 / (1 + exp((eps - mu) / sigma)), sigma = k_B T.
* ``fermi_level``          -- Alg. 5 step 1: the mu at which
  2 (N_oc + sum_{fr} f(eps_k, mu)) = N_e, by Brent's method on that monotone
  function (scipy ``brentq``).
* ``projected_split``      -- the mixed-precision projected Hamiltonian of
  Sec. 3.5 (eq. partialDiagMixedPrec1): the fr-fr block in FP64, every other
  block from FP32 inputs with FP32 products.
* ``rayleigh_ritz_split``  -- Alg. 4: Hhat = X^T Htilde X (FP64, or the mixed
  form above), all eigenpairs of Hhat, the N_fr largest kept, the partial
  rotation X_fr = X Q_fr and its residual norms.
* ``density_split``        -- Alg. 5 steps 2-3, eq. elecDensSP: with the
  collocated GLL quadrature (the basis functions are the Lagrange polynomials
  of the nodes, so n^e(x_j) is the unit vector of node j) the density at node
  j is 2 M_jj^-1 ( sum_i X[j,i]^2 + sum_k (f(eps_k, mu) - 1) X_fr[j,k]^2 ).
* ``density_full``         -- eq. elecDens: the same density from a full
  rotation, 2 M_jj^-1 sum_i f_i (X Q)[j,i]^2 with f_i = 1 for the N_oc lowest
  pairs (the paper's f(D_oc, mu) = I) and f(eps_i, mu) for the rest.
* ``density_cellwise``     -- eq. elecDensSums evaluated literally: for every
  cell and each of its GLL nodes, the wavefunctions interpolated through the
  cell's tensor-product Lagrange basis (``fem.lagrange_eval``).  Slow; for
  tiny meshes only.

Pins (tests/test_oracle_density.py): the Fermi-Dirac symmetry
f(mu + d) + f(mu - d) = 1; mu for two levels and for a spectrum symmetric
about mu0 (closed forms); the particle count sum_j M_jj rho_j = N_e; split
against full (the projector identity X X^T = X Q Q^T X^T); the cell-level
formula against the nodal one on every cell; the particle-in-a-box ground
state density against the separable product of 1D eigenvectors; the FP64
``rayleigh_ritz_split`` against the top N_fr pairs of the full Rayleigh-Ritz;
``projected_split`` against exactly rounded sums (``math.fsum``: FP64-level
error in the fr-fr block, FP32-level error outside it) and bit-exact where
FP32 arithmetic is exact; the mixed split on exact eigenvectors, where the
coupling blocks vanish, against the exact eigenvalues to FP64 level (the
paper's limit, eq. partialDiagLim2), and on a random block with an error
between FP32-level bounds.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize as so

from . import fem


def fermi_dirac(eps, mu: float, sigma: float):
    """Occupancy in [0, 1] (Sec. 2.1); sigma > 0."""
    x = (np.asarray(eps, dtype=np.float64) - mu) / sigma
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(x))


def electron_count(evals_fr, n_oc: int, mu: float, sigma: float) -> float:
    """2 (N_oc + sum_k f(eps_k, mu)), the left side of Alg. 5 step 1."""
    return 2.0 * (n_oc + float(np.sum(fermi_dirac(evals_fr, mu, sigma))))


def fermi_level(evals_fr, n_oc: int, n_electrons: float, sigma: float) -> float:
    """The Fermi energy of Alg. 5 step 1.  The count rises monotonically from
    2 N_oc (mu -> -inf) to 2 (N_oc + N_fr) (mu -> +inf); N_e must lie strictly
    between them."""
    e = np.asarray(evals_fr, dtype=np.float64)
    lo_n, hi_n = 2.0 * n_oc, 2.0 * (n_oc + e.size)
    if not (lo_n < n_electrons < hi_n):
        raise ValueError(f"N_e = {n_electrons} outside ({lo_n}, {hi_n})")
    g = lambda mu: electron_count(e, n_oc, mu, sigma) - n_electrons
    a, b = float(e.min()), float(e.max())
    while g(a) > 0:
        a -= 10.0 * sigma + (b - a)
    while g(b) < 0:
        b += 10.0 * sigma + (b - a)
    return float(so.brentq(g, a, b, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500))


def projected_split(X: np.ndarray, HX: np.ndarray, fr0: int) -> np.ndarray:
    """G = X^T HX as in eq. partialDiagMixedPrec1 (Sec. 3.5): the block of rows
    and columns >= fr0 (the fractionally occupied states) in FP64, every other
    entry from inputs rounded to FP32 with FP32 products and sums."""
    G = (X.astype(np.float32).T @ HX.astype(np.float32)).astype(np.float64)
    G[fr0:, fr0:] = X[:, fr0:].T @ HX[:, fr0:]
    return G


def rayleigh_ritz_split(apply, X: np.ndarray, n_fr: int, mixed: bool = False, fr0: int | None = None):
    """Alg. 4 on an orthonormal X [n x N].  Returns (X_fr = X Q_fr, D_fr, resid).

    mixed: Hhat by ``projected_split`` with the FP64 block starting at fr0
    (default N - n_fr); otherwise all FP64."""
    N = X.shape[1]
    HX = apply(X)
    if fr0 is None:
        fr0 = N - n_fr
    G = projected_split(X, HX, fr0) if mixed else X.T @ HX
    Hhat = np.tril(G) + np.tril(G, -1).T
    D, Q = np.linalg.eigh(Hhat)
    Qfr = Q[:, N - n_fr:]
    Xfr = X @ Qfr
    HXfr = HX @ Qfr
    Dfr = D[N - n_fr:]
    res = np.linalg.norm(HXfr - Xfr * Dfr[None, :], axis=0)
    return Xfr, Dfr, res


def density_split(X: np.ndarray, Xfr: np.ndarray, evals_fr, mu: float, sigma: float,
                  minv: np.ndarray) -> np.ndarray:
    """Nodal density by eq. elecDensSP; minv = M^-1/2 per DoF."""
    w = fermi_dirac(evals_fr, mu, sigma) - 1.0
    s = np.sum(X * X, axis=1) + (Xfr * Xfr) @ w
    return 2.0 * minv * minv * s


def density_full(Xr: np.ndarray, evals, n_oc: int, mu: float, sigma: float,
                 minv: np.ndarray) -> np.ndarray:
    """Nodal density by eq. elecDens from fully rotated Ritz vectors Xr."""
    f = np.ones(Xr.shape[1])
    f[n_oc:] = fermi_dirac(np.asarray(evals)[n_oc:], mu, sigma)
    return 2.0 * minv * minv * ((Xr * Xr) @ f)


def density_cellwise(L: float, n_el: int, p: int, Xr: np.ndarray, occ: np.ndarray,
                     minv: np.ndarray) -> np.ndarray:
    """eq. elecDensSums at each cell's GLL nodes: rho(x) = 2 sum_i f_i
    (sum_j psi_i^{e,j} N_j^e(x))^2 with psi = M^-1/2 X (zero at Dirichlet
    nodes) and N^e the tensor-product Lagrange basis.  Returns [n_cells x
    (p+1)^3] values, local node order a + (p+1) b + (p+1)^2 c."""
    xi, _ = fem.gll(p)
    B = fem.lagrange_eval(xi, xi)                 # B[q, a] = l_a(xi_q)
    cmap = fem.cell_dof_map(n_el, p)
    psi = np.vstack([minv[:, None] * Xr, np.zeros((1, Xr.shape[1]))])  # row -1 -> 0
    n1 = p + 1
    out = np.zeros((cmap.shape[0], n1 ** 3))
    for e in range(cmap.shape[0]):
        g = np.where(cmap[e] >= 0, cmap[e], psi.shape[0] - 1)
        P = psi[g].reshape(n1, n1, n1, -1)        # [c, b, a, state]
        # interpolate to the nodes through the basis in each direction
        vals = np.einsum("zc,yb,xa,cbas->zyxs", B, B, B, P)
        out[e] = 2.0 * ((vals.reshape(n1 ** 3, -1) ** 2) @ occ)
    return out


__all__ = ["fermi_dirac", "electron_count", "fermi_level", "projected_split", "rayleigh_ritz_split", "density_split",
           "density_full", "density_cellwise"]
