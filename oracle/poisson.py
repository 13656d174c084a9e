"""Oracle: the discrete Poisson problem of the electrostatics, FP64 on the CPU.
TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2.4 eq. phiTotDiscreteSolve, homogeneous Dirichlet conditions on
[0, L]^3 (the non-periodic case):

    sum_j [ 1/(4 pi) int grad N_i . grad N_j ] phi_j = int (rho + b) N_i,

on the same GLL spectral elements.  With the GLL rule collocated at the nodes
the right-hand side of a nodal density is M rho (M the diagonal mass), and a
point charge q sitting on node i (the paper places nuclear charges on nodes,
b_I = -Z_I delta) contributes q to entry i.  The Laplacian stiffness is twice
``fem.assemble``'s (which is that of -1/2 Laplacian), so the system matrix is
A = K_half / (2 pi).

* ``poisson_matrix`` / ``load_vector`` / ``solve``  -- the plain definition:
  assemble and solve directly (sparse LU);
* ``jacobi_pcg``  -- the paper's solver (Sec. 3.2): conjugate gradients with
  the diagonal (Jacobi) preconditioner, in its textbook form (Shewchuk), with
  the relative residual ||f - A phi|| / ||f|| as the stopping rule.

Pins (tests/test_oracle_poisson.py): the manufactured solution
phi = sin(pi x/L) sin(pi y/L) sin(pi z/L), for which rho = 3 pi phi / (4 L^2),
is reproduced with spectral accuracy (error falling with p); A is symmetric
positive definite and equals the Kronecker sum of 1D operators; PCG reaches
the direct solution; point charges obey reciprocity (the potential at j of a
unit charge on i equals that at i of one on j, which a charge scaled by the
nodal mass would break) and superpose.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


def poisson_matrix(L: float, n_el: int, p: int):
    """(A, M): A = 1/(4 pi) int grad N_i . grad N_j (CSR, interior DoFs), M the
    diagonal GLL mass."""
    K, M = fem.assemble(L, n_el, p)
    return (K * (1.0 / (2.0 * np.pi))).tocsr(), M


def load_vector(M: np.ndarray, rho: np.ndarray, charge_dofs=(), charges=()) -> np.ndarray:
    """int (rho + b) N_i with the GLL rule: M rho, plus each point charge on its node."""
    f = M * np.asarray(rho, dtype=np.float64)
    for d, q in zip(charge_dofs, charges):
        f[int(d)] += float(q)
    return f


def solve(L: float, n_el: int, p: int, rho, charge_dofs=(), charges=()) -> np.ndarray:
    """phi from A phi = M rho + q by a sparse direct solve (the plain definition)."""
    A, M = poisson_matrix(L, n_el, p)
    return spla.spsolve(A.tocsc(), load_vector(M, rho, charge_dofs, charges))


def jacobi_pcg(A, f: np.ndarray, tol: float = 1e-10, max_iter: int = 10000, x0=None):
    """Conjugate gradients preconditioned by diag(A).  Returns (x, iterations,
    relative residual history)."""
    d = A.diagonal()
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - A @ x
    z = r / d
    pvec = z.copy()
    rz = r @ z
    fn = np.linalg.norm(f)
    hist = [np.linalg.norm(r) / fn]
    it = 0
    while hist[-1] > tol and it < max_iter:
        q = A @ pvec
        alpha = rz / (pvec @ q)
        x += alpha * pvec
        r -= alpha * q
        z = r / d
        rz_new = r @ z
        hist.append(np.linalg.norm(r) / fn)
        pvec = z + (rz_new / rz) * pvec
        rz = rz_new
        it += 1
    return x, it, hist


def manufactured(L: float, xyz: np.ndarray):
    """(phi, rho) with phi = prod sin(pi x_d / L) (zero on the walls) and
    rho = -(1/4pi) Laplacian phi = 3 pi phi / (4 L^2)."""
    phi = np.prod(np.sin(np.pi * xyz / L), axis=1)
    return phi, 3.0 * np.pi * phi / (4.0 * L * L)


__all__ = ["poisson_matrix", "load_vector", "solve", "jacobi_pcg", "manufactured"]
