"""Oracle: Chebyshev-filtered subspace iteration steps, FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``cheb_filter_paper``   -- the paper's three-term recursion
  T_m(Hbar) X = [2 Hbar T_{m-1}(Hbar) - T_{m-2}(Hbar)] X with
  Hbar = (Htilde - c)/e mapping the unwanted interval [a, b] onto [-1, 1]
  (Sec. 3.3, eq. chebFilter).
* ``cheb_filter_scaled``  -- the same polynomial divided by T_m(xi0),
  xi0 = (a0 - c)/e, evaluated through the normalised recursion (ratios
  rho_k = t_{k-1}/t_k of the scalar sequence t_k = T_k(xi0)).  Equal to
  ``cheb_filter_paper(...) / T_m(xi0)`` in exact arithmetic.
* ``cholgs``              -- Sec. 3.4 Alg. 3: S = X^T X, S = L L^T, L^-1,
  X_o = X L^-T.
* ``cholgs_mixed``        -- Sec. 3.4 eq. overlapmixedprec: diagonal blocks
  of S and of L^-T in FP64, off-diagonal blocks with FP32 inputs and FP32
  accumulation (``overlap_mixed``, ``rmul_mixed``).  (The paper splits off
  diagonal *entries*; block width 1 is that case.)
* ``rayleigh_ritz``       -- Sec. 3.5 steps i-iii: Hhat = X^T Htilde X (lower
  triangle, mirrored), Hhat Q = Q D with D ascending, X <- X Q; also
  HX <- HX Q and the residual norms ||HX_i - D_i X_i||.
* ``chfsi_solve``         -- Alg. 2 step 7 with the adaptive repeat of
  Sec. 3.3: CholGS + RR on the start block, then {filter, CholGS, RR} until the
  largest residual of the wanted states is <= tol.
* ``eig_dense`` / ``eig_lanczos`` -- the plain definition of the result: the
  lowest eigenpairs of Htilde by LAPACK (numpy ``eigh``) or ARPACK Lanczos.
* ``cheb_T``, ``filter_coefficients`` -- T_m(x) by its closed form, and the
  (s1, s2, shift) of each step of the normalised recursion (Sec. 3.3).
* ``subspace_angle``, ``cluster_boundaries`` -- comparison helpers of the tests
  (largest principal angle; the counts at which the spectrum has a gap), not
  steps of the method.

Pins (tests/test_oracle_chfsi.py): the filter against the closed form
T_m(x) = cos(m arccos x) / cosh(m arccosh |x|) on exact eigenvectors and the
two recursions against each other; CholGS against Householder QR with a
positive R diagonal; the mixed split against exactly rounded sums
(``math.fsum``): FP64-level error on the diagonal blocks, an error inside the
FP32 accumulation bound and far above FP64 rounding off them, bit-exact
results where FP32 arithmetic is exact (small integers), and FP64 equality
when the off-diagonal blocks vanish; RR on rotated exact eigenvectors; the solve loop against
dense ``eigh``; dense against Lanczos; T_m's closed form against its
recurrence; the step coefficients against the scaled filter; the subspace
angle against the planar closed form and scipy's principal angles.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


# --------------------------------------------------------------------------
# Chebyshev filter (Sec. 3.3)
# --------------------------------------------------------------------------

def cheb_T(m: int, x):
    """Closed form of the Chebyshev polynomial of the first kind."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** m * np.cosh(m * np.arccosh(np.abs(xo)))
    return out


def cheb_filter_paper(apply, X: np.ndarray, m: int, a: float, b: float) -> np.ndarray:
    """Y_m = T_m(Hbar) X by Y_{k+1} = 2 Hbar Y_k - Y_{k-1}, Y_0 = X, Y_1 = Hbar X."""
    c, e = 0.5 * (a + b), 0.5 * (b - a)
    hbar = lambda Y: (apply(Y) - c * Y) / e
    if m == 0:
        return X.copy()
    y_prev, y = X.copy(), hbar(X)
    for _ in range(1, m):
        y_prev, y = y, 2.0 * hbar(y) - y_prev
    return y


def cheb_filter_scaled(apply, X: np.ndarray, m: int, a: float, b: float, a0: float) -> np.ndarray:
    """Z_m = T_m(Hbar) X / T_m(xi0).

    With rho_1 = 1/xi0 and rho_{k+1} = 1/(2 xi0 - rho_k) (rho_k = t_{k-1}/t_k):
    Z_1 = rho_1 Hbar X,  Z_{k+1} = 2 rho_{k+1} Hbar Z_k - rho_{k+1} rho_k Z_{k-1}.
    """
    c, e = 0.5 * (a + b), 0.5 * (b - a)
    xi0 = (a0 - c) / e
    hbar = lambda Y: (apply(Y) - c * Y) / e
    if m == 0:
        return X.copy()
    rho = 1.0 / xi0
    z_prev, z = X.copy(), rho * hbar(X)
    for _ in range(1, m):
        rho_next = 1.0 / (2.0 * xi0 - rho)
        z_prev, z = z, 2.0 * rho_next * hbar(z) - rho_next * rho * z_prev
        rho = rho_next
    return z


def filter_coefficients(m: int, a: float, b: float, a0: float):
    """Per-step (sigma1, sigma2, shift) such that step k computes
    Z_{k+1} = sigma1 (Htilde - shift) Z_k + sigma2 Z_{k-1}; same recursion as
    ``cheb_filter_scaled``.  Used by tests to drive single GPU steps."""
    c, e = 0.5 * (a + b), 0.5 * (b - a)
    xi0 = (a0 - c) / e
    out = []
    rho = 1.0 / xi0
    out.append((rho / e, 0.0, c))
    for _ in range(1, m):
        rho_next = 1.0 / (2.0 * xi0 - rho)
        out.append((2.0 * rho_next / e, -rho_next * rho, c))
        rho = rho_next
    return out


# --------------------------------------------------------------------------
# CholGS (Sec. 3.4, Alg. 3)
# --------------------------------------------------------------------------

class NotSPD(ArithmeticError):
    pass


def cholgs(X: np.ndarray) -> np.ndarray:
    """Steps 1-4 of Alg. 3 in FP64; returns X_o with X_o^T X_o = I."""
    S = X.T @ X                                   # step 1
    try:
        L = np.linalg.cholesky(S)                 # step 2: S = L L^T
    except np.linalg.LinAlgError as exc:
        raise NotSPD(str(exc)) from exc
    Linv = sla.solve_triangular(L, np.eye(L.shape[0]), lower=True)   # step 3
    return X @ Linv.T                             # step 4


def _block_masks(n: int, bv: int):
    blk = np.arange(n) // bv
    diag = blk[:, None] == blk[None, :]
    return diag


def overlap_mixed(X: np.ndarray, bv: int = 64) -> np.ndarray:
    """Step 1 of Alg. 3 split as in eq. overlapmixedprec: S = X^T X with the
    bv x bv diagonal blocks in FP64 and every off-diagonal block from inputs
    rounded to FP32 (nearest) with FP32 products and sums, promoted to FP64."""
    n = X.shape[1]
    diag = _block_masks(n, bv)
    X32 = X.astype(np.float32)
    return np.where(diag, X.T @ X, (X32.T @ X32).astype(np.float64))


def rmul_mixed(X: np.ndarray, U: np.ndarray, bv: int = 64) -> np.ndarray:
    """Step 4 of Alg. 3 split the same way (the product after eq.
    overlapmixedprec): X U with the bv x bv diagonal blocks of U applied in
    FP64 and the off-diagonal blocks with FP32 inputs, products and sums."""
    n = U.shape[0]
    diag = _block_masks(n, bv)
    Ud = np.where(diag, U, 0.0)
    Uod = np.where(diag, 0.0, U).astype(np.float32)
    return X @ Ud + (X.astype(np.float32) @ Uod).astype(np.float64)


def cholgs_mixed(X: np.ndarray, bv: int = 64) -> np.ndarray:
    """Alg. 3 with the mixed-precision split of steps 1 and 4 (``overlap_mixed``
    and ``rmul_mixed``); steps 2 and 3 (Cholesky factor and its inverse) in
    FP64, as in the paper."""
    n = X.shape[1]
    S = overlap_mixed(X, bv)
    try:
        L = np.linalg.cholesky(S)
    except np.linalg.LinAlgError as exc:
        raise NotSPD(str(exc)) from exc
    U = sla.solve_triangular(L, np.eye(n), lower=True).T      # L^-T, upper
    return rmul_mixed(X, U, bv)


# --------------------------------------------------------------------------
# Rayleigh-Ritz (Sec. 3.5)
# --------------------------------------------------------------------------

def rayleigh_ritz(apply, X: np.ndarray):
    """Returns (X Q, HX Q, D ascending, residual norms)."""
    HX = apply(X)
    G = X.T @ HX
    Hhat = np.tril(G) + np.tril(G, -1).T          # lower triangle, mirrored
    D, Q = np.linalg.eigh(Hhat)
    Xr = X @ Q
    HXr = HX @ Q
    res = np.linalg.norm(HXr - Xr * D[None, :], axis=0)
    return Xr, HXr, D, res


# --------------------------------------------------------------------------
# Subspace iteration loop
# --------------------------------------------------------------------------

def chfsi_solve(apply, X0: np.ndarray, nstates: int, degree: int, b: float,
                tol: float, max_iter: int = 200, mixed: bool = False):
    """ChFSI: CholGS + RR on X0; then repeat {filter with a = largest Ritz value,
    a0 = smallest Ritz value; CholGS; RR} until max_{i<=nstates} r_i <= tol.

    Returns dict(evals, evecs, resid, iters, converged)."""
    orth = cholgs_mixed if mixed else cholgs
    X = orth(X0)
    X, _, D, r = rayleigh_ritz(apply, X)
    it = 0
    while np.max(r[:nstates]) > tol and it < max_iter:
        X = cheb_filter_scaled(apply, X, degree, float(D[-1]), b, float(D[0]))
        X = orth(X)
        X, _, D, r = rayleigh_ritz(apply, X)
        it += 1
    return dict(evals=D, evecs=X, resid=r, iters=it, converged=bool(np.max(r[:nstates]) <= tol))


# --------------------------------------------------------------------------
# The plain definition: eigenpairs of Htilde
# --------------------------------------------------------------------------

def eig_dense(H) -> tuple:
    """All eigenpairs of the symmetric H, ascending (LAPACK through numpy)."""
    H = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    return np.linalg.eigh(H)


def eig_lanczos(apply, n: int, k: int, tol: float = 1e-13, seed: int = 7):
    """Lowest k eigenpairs by ARPACK (implicitly restarted Lanczos)."""
    op = spla.LinearOperator((n, n), matvec=lambda v: apply(v.reshape(-1)), dtype=np.float64)
    v0 = np.random.Generator(np.random.PCG64(seed)).standard_normal(n)
    w, v = spla.eigsh(op, k=k, which="SA", tol=tol, v0=v0, ncv=max(2 * k + 1, 20))
    order = np.argsort(w)
    return w[order], v[:, order]


# --------------------------------------------------------------------------
# Comparison helpers (what is unique in an eigen-result)
# --------------------------------------------------------------------------

def subspace_angle(A: np.ndarray, B: np.ndarray) -> float:
    """Largest principal angle between span(A) and span(B), both with orthonormal
    columns and the same count: arcsin ||B - A (A^T B)||_2 (the sine form stays
    accurate for small angles, where arccos of the cosines cannot go below ~1e-8)."""
    Q, _ = np.linalg.qr(A)
    Bq, _ = np.linalg.qr(B)
    R = Bq - Q @ (Q.T @ Bq)
    s = np.linalg.norm(R, 2) if R.size else 0.0
    return float(np.arcsin(min(1.0, s)))


def cluster_boundaries(evals: np.ndarray, upto: int, gap: float = 1e-3):
    """Indices k (1-based counts) <= upto at which evals[k] - evals[k-1] >= gap."""
    return [k for k in range(1, min(upto, evals.shape[0] - 1) + 1)
            if evals[k] - evals[k - 1] >= gap]


__all__ = ["cheb_T", "cheb_filter_paper", "cheb_filter_scaled", "filter_coefficients",
           "NotSPD", "cholgs", "overlap_mixed", "rmul_mixed", "cholgs_mixed", "rayleigh_ritz", "chfsi_solve", "eig_dense",
           "eig_lanczos", "subspace_angle", "cluster_boundaries"]
