"""Oracle: Chebyshev-filtered subspace iteration on the complex Hermitian
Bloch operator at a k-point, complex128 on the CPU.  TEST INFRASTRUCTURE ONLY
(see ``oracle/__init__``).

At k != 0 the standard-form operator Htilde_k of eq. ksproblemPer (Sec. 2.1;
``kpoint.htilde_k_csr``) is complex Hermitian, so every step of the method
(Sec. 3.3 - 3.5) takes its Hermitian form: overlaps and projections use the
conjugate transpose, the Cholesky factor of X^H X is complex lower triangular
with a positive real diagonal, and the projected eigenproblem is Hermitian.
The Chebyshev filter has real coefficients and is the same recursion on
complex blocks (``chfsi.cheb_filter_scaled`` applies unchanged).

* ``cholgs_c``          -- Alg. 3 in complex arithmetic: S = X^H X, S = L L^H,
  X_o = X L^-H.
* ``rayleigh_ritz_c``   -- Sec. 3.5 steps i-iii: Hhat = X^H Htilde_k X (lower
  triangle, completed by Hermitian symmetry), Hhat Q = Q D (D ascending),
  X <- X Q, HX <- HX Q, residual norms.
* ``chfsi_solve_c``     -- the loop of ``chfsi.chfsi_solve`` on these steps.
* ``upper_bound_k``     -- lambda_max(Htilde_k) <= sum_d lambda_max(A_{k_d}) +
  max V (Weyl: Htilde_k is the Kronecker sum of the three 1D Bloch operators
  plus a diagonal).

Pins (tests/test_oracle_kchfsi.py): CholGS against complex Householder QR with
the phases of R's diagonal removed; X^H X = I; Rayleigh-Ritz on exact Bloch
eigenvectors (tensor products of 1D eigenvectors) mixed by a random unitary
returns their exact eigenvalues; the solve against the dense Hermitian
eigensolve of ``kpoint.htilde_k_csr`` (eigenvalues 1e-10 relative, subspace
angles 1e-8 at cluster boundaries) and, at V = 0, against sums of 1D Bloch
eigenvalues; the bound against the dense largest eigenvalue; the filter on
exact eigenvectors against the closed form T_m.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .chfsi import NotSPD, cheb_filter_scaled


def cholgs_c(X: np.ndarray) -> np.ndarray:
    """Steps 1-4 of Alg. 3 on a complex block; returns X_o with X_o^H X_o = I."""
    S = X.conj().T @ X
    try:
        L = np.linalg.cholesky(S)                 # S = L L^H, L lower, real positive diagonal
    except np.linalg.LinAlgError as exc:
        raise NotSPD(str(exc)) from exc
    Linv = sla.solve_triangular(L, np.eye(L.shape[0], dtype=np.complex128), lower=True)
    return X @ Linv.conj().T


def rayleigh_ritz_c(apply, X: np.ndarray):
    """Returns (X Q, HX Q, D ascending, residual norms) for orthonormal complex X."""
    HX = apply(X)
    G = X.conj().T @ HX
    Hhat = np.tril(G) + np.tril(G, -1).conj().T
    Hhat[np.diag_indices_from(Hhat)] = Hhat.diagonal().real
    D, Q = np.linalg.eigh(Hhat)
    Xr = X @ Q
    HXr = HX @ Q
    res = np.linalg.norm(HXr - Xr * D[None, :], axis=0)
    return Xr, HXr, D, res


def chfsi_solve_c(apply, X0: np.ndarray, nstates: int, degree: int, b: float, tol: float, max_iter: int = 200):
    """CholGS + RR on X0, then {filter with a = largest, a0 = smallest Ritz
    value; CholGS; RR} until max_{i < nstates} r_i <= tol."""
    X = cholgs_c(np.asarray(X0, dtype=np.complex128))
    X, _, D, r = rayleigh_ritz_c(apply, X)
    it = 0
    while np.max(r[:nstates]) > tol and it < max_iter:
        X = cheb_filter_scaled(apply, X, degree, float(D[-1]), b, float(D[0]))
        X = cholgs_c(X)
        X, _, D, r = rayleigh_ritz_c(apply, X)
        it += 1
    return dict(evals=D, evecs=X, resid=r, iters=it, converged=bool(np.max(r[:nstates]) <= tol))


def upper_bound_k(Ax: np.ndarray, Ay: np.ndarray, Az: np.ndarray, V: np.ndarray) -> float:
    return float(sum(np.linalg.eigvalsh(A)[-1] for A in (Ax, Ay, Az)) + np.max(V))


__all__ = ["cholgs_c", "rayleigh_ritz_c", "chfsi_solve_c", "upper_bound_k"]
