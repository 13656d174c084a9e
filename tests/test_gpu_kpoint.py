"""GPU parity of the periodic mesh and the complex Bloch operator (Sec. 2.1,
eq. ksproblemPer) against the oracle."""
import numpy as np
import pytest

import paper_1903_10959_amd as P
from oracle import kpoint
import workload

pytestmark = pytest.mark.gpu


def _ctx(L, n_el, p, k, seed=8, nwells=2):
    c = P.Context(0).set_mesh(L, n_el, p, periodic=True)
    V = workload.eval_wells(workload.draw_wells(nwells, L, seed, (1.0, 2.0), (0.3, 0.6)), c.dof_coords())
    c.set_potential(V)
    c.set_kpoint(k)
    return c, V


def _cgpu(X, ld=None):
    import torch
    X = np.asarray(X, dtype=np.complex128)
    if ld is None or ld == X.shape[1]:
        return torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")
    buf = torch.zeros((X.shape[0], ld), dtype=torch.complex128, device="cuda:0")
    buf[:, :X.shape[1]] = torch.from_numpy(X).to("cuda:0")
    return buf[:, :X.shape[1]]


def _rand(n, c, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, c)) + 1j * rng.standard_normal((n, c))


KS = [(0.0, 0.0, 0.0), (0.31, -0.52, 0.11), (1.3, 0.0, -0.7)]


@pytest.mark.parametrize("L,n_el,p", [(5.0, 2, 1), (5.0, 2, 3), (6.0, 2, 4), (8.0, 4, 4), (6.0, 2, 5), (7.0, 2, 6),
                                      (7.0, 2, 7)])
@pytest.mark.parametrize("ki", [0, 1, 2])
def test_apply_complex_matches_oracle(L, n_el, p, ki):
    k = np.array(KS[ki])
    c, V = _ctx(L, n_el, p, k)
    H = kpoint.htilde_k_csr(L, n_el, p, V, k)
    for ncols, ld in ((1, 1), (5, 7), (33, 33), (40, 45)):
        X = _rand(c.n_dof, ncols, 100 + ncols)
        Y = c.apply_complex(_cgpu(X, ld)).cpu().numpy()
        Yo = H @ X
        err = np.max(np.abs(Y - Yo)) / np.max(np.abs(Yo))
        assert err < 1e-13, (ncols, ld, err)
    c.close()


def test_apply_complex_at_gamma_equals_real_apply():
    import torch
    c, V = _ctx(6.0, 2, 4, (0.0, 0.0, 0.0))
    X = _rand(c.n_dof, 24, 3)
    Yc = c.apply_complex(_cgpu(X)).cpu().numpy()
    Xr = torch.from_numpy(np.ascontiguousarray(X.real)).to("cuda:0")
    Xi = torch.from_numpy(np.ascontiguousarray(X.imag)).to("cuda:0")
    Yr = c.apply(Xr).cpu().numpy()
    Yi = c.apply(Xi).cpu().numpy()
    np.testing.assert_allclose(Yc, Yr + 1j * Yi, rtol=0, atol=1e-14 * np.abs(Yc).max())
    c.close()


def test_apply_complex_is_hermitian():
    """x2^H (H x1) = (H x2)^H x1 for random blocks (a property at any size)."""
    c, _ = _ctx(8.0, 4, 5, (0.4, 0.9, -0.2))
    X1, X2 = _rand(c.n_dof, 8, 1), _rand(c.n_dof, 8, 2)
    Y1 = c.apply_complex(_cgpu(X1)).cpu().numpy()
    Y2 = c.apply_complex(_cgpu(X2)).cpu().numpy()
    a, b = X2.conj().T @ Y1, Y2.conj().T @ X1
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()
    c.close()


def test_gamma_point_solve_on_periodic_mesh():
    """The real ChFSI path on the periodic mesh (k = 0) reaches the lowest
    eigenvalues of the oracle's periodic operator (dense eigh)."""
    import torch
    L, n_el, p = 6.0, 2, 4
    c, V = _ctx(L, n_el, p, (0.0, 0.0, 0.0), nwells=3)
    ev = np.linalg.eigvalsh(kpoint.htilde_k_csr(L, n_el, p, V, [0, 0, 0]).toarray())
    N = 8
    while ev[N] - ev[N - 1] < 1e-6:
        N += 1
    nb = workload.block_size(N)
    X = torch.from_numpy(workload.start_block(c.n_dof, nb, 5)).to("cuda:0")
    out = c.solve(X, N, 20, 1e-9 * max(1.0, abs(ev[0])), max_iter=300)
    assert out["converged"]
    np.testing.assert_allclose(out["evals"][:N], ev[:N], rtol=1e-10, atol=1e-10)
    c.close()


def test_kpoint_group_equals_single_applies():
    """A group of k-points in one launch per colour gives each k-point's own
    apply (padded row stride and a block stride beyond n_dof * ld)."""
    import torch
    L, n_el, p = 6.0, 2, 4
    ks = np.array([[0.0, 0.0, 0.0], [0.26, 0.26, 0.0], [0.26, -0.26, 0.52], [-0.7, 0.1, 0.3]])
    c, V = _ctx(L, n_el, p, (0.0, 0.0, 0.0))
    c.set_kpoints(ks)
    nk, ncols = ks.shape[0], 33
    big = torch.zeros((nk, c.n_dof + 3, 40), dtype=torch.complex128, device="cuda:0")
    Xh = np.stack([_rand(c.n_dof, ncols, 50 + g) for g in range(nk)])
    big[:, :c.n_dof, :ncols] = torch.from_numpy(Xh).to("cuda:0")
    X = big[:, :c.n_dof, :ncols]
    Y = c.apply_complex_kpoints(X).cpu().numpy()
    for g in range(nk):
        c.set_kpoint(ks[g])
        Yg = c.apply_complex(_cgpu(Xh[g])).cpu().numpy()
        np.testing.assert_allclose(Y[g], Yg, rtol=0, atol=1e-15 * np.abs(Yg).max())
    Yo = kpoint.htilde_k_csr(L, n_el, p, V, ks[-1]) @ Xh[-1]
    assert np.max(np.abs(Y[-1] - Yo)) < 1e-13 * np.max(np.abs(Yo))
    c.close()
