"""GPU parity of ChFSI on the complex Bloch operator at k != 0 (Sec. 2.1 eq.
ksproblemPer; the Hermitian forms of Sec. 3.3 - 3.5) against the oracle
(oracle/kchfsi.py, oracle/kpoint.py)."""
import numpy as np
import pytest

from oracle import chfsi as och
from oracle import kchfsi, kpoint
import workload

pytestmark = pytest.mark.gpu

K = np.array([0.13, -0.21, 0.08])


def _ctx(L, n_el, p, k=K, wells=True, seed=8):
    import paper_1903_10959_amd as P
    c = P.Context(0).set_mesh(L, n_el, p, periodic=True)
    if wells:
        V = workload.eval_wells(workload.draw_wells(max(3, int(L ** 3 / 1000)), L, seed, (1.0, 3.0), (0.5, 1.0)),
                                c.dof_coords())
    else:
        V = np.zeros(c.n_dof)
    c.set_potential(V)
    c.set_kpoint(k)
    A = [kpoint.operator_1d_periodic(L, n_el, p, kd) for kd in k]
    return c, V, A, (lambda Y: kpoint.apply_kron_k(*A, V, Y))


def _gpu(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex128))).to("cuda:0")


def _host(t):
    return t.detach().cpu().numpy()


def _cblock(n, m, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))


def test_upper_bound_k_matches_the_oracle_and_bounds_the_spectrum():
    L, n_el, p = 6.0, 2, 4
    c, V, A, _ = _ctx(L, n_el, p)
    b_o = kchfsi.upper_bound_k(*A, V)
    assert abs(c.upper_bound_k - b_o) < 1e-10 * b_o
    lmax = np.linalg.eigvalsh(kpoint.htilde_k_csr(L, n_el, p, V, K).toarray())[-1]
    assert c.upper_bound_k >= lmax
    c.close()


@pytest.mark.parametrize("ncols,decades", [(24, 2), (65, 1), (130, 1)])
def test_orthonormalize_complex_matches_householder(ncols, decades):
    c, V, A, _ = _ctx(8.0, 4, 4)
    X = _cblock(c.n_dof, ncols, ncols) @ np.diag(np.logspace(0, decades, ncols))
    Xg = _gpu(X)
    c.orthonormalize_complex(Xg)
    Xo = _host(Xg)
    Q, R = np.linalg.qr(X)
    Q = Q * (np.diag(R) / np.abs(np.diag(R)))[None, :]
    kappa = np.linalg.cond(X)
    assert np.max(np.abs(Xo - Q)) < 1e-13 * kappa ** 2
    assert np.max(np.abs(Xo.conj().T @ Xo - np.eye(ncols))) < 1e-13 * kappa ** 2
    np.testing.assert_allclose(Xo, kchfsi.cholgs_c(X), rtol=0, atol=1e-13 * kappa ** 2)
    c.close()


@pytest.mark.parametrize("ncols", [1, 7, 33, 64, 100])
def test_rayleigh_ritz_complex_matches_oracle(ncols):
    c, V, A, ap = _ctx(8.0, 4, 4)
    X = kchfsi.cholgs_c(_cblock(c.n_dof, ncols, 100 + ncols))
    Xr, HXr, D, res = kchfsi.rayleigh_ritz_c(ap, X)
    Xg = _gpu(X)
    HX = _gpu(np.zeros_like(X))
    ev, rs = c.rayleigh_ritz_complex(Xg, HX_out=HX)
    assert c.last_eigensolve_converged
    scale = max(1.0, np.max(np.abs(D)))
    np.testing.assert_allclose(ev, D, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(rs, res, rtol=1e-6, atol=1e-11 * scale)
    G = _host(Xg)
    assert np.max(np.abs(_host(HX) - ap(G))) < 1e-11 * scale
    assert np.max(np.abs(G.conj().T @ G - np.eye(ncols))) < 1e-12
    # Ritz vectors up to a phase (the projected spectrum of a random block is simple)
    ov = np.abs(np.sum(G.conj() * Xr, axis=0))
    np.testing.assert_allclose(ov, 1.0, atol=1e-8)
    c.close()


def test_rayleigh_ritz_complex_exact_on_bloch_eigenvectors():
    """Exact eigenvectors of the V = 0 Bloch operator (tensor products of 1D
    eigenvectors), mixed by a random unitary: their exact eigenvalues."""
    L, n_el, p = 8.0, 4, 3
    c, V, A, ap = _ctx(L, n_el, p, wells=False)
    eig = [np.linalg.eigh(a) for a in A]
    picks = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (2, 0, 0), (3, 1, 1), (2, 2, 2), (5, 4, 0),
             (0, 6, 7)]
    X = np.stack([np.kron(eig[2][1][:, l], np.kron(eig[1][1][:, j], eig[0][1][:, i])) for (i, j, l) in picks], 1)
    lam = np.array([eig[0][0][i] + eig[1][0][j] + eig[2][0][l] for (i, j, l) in picks])
    U, _ = np.linalg.qr(_cblock(len(picks), len(picks), 5))
    ev, rs = c.rayleigh_ritz_complex(_gpu(X @ U))
    np.testing.assert_allclose(ev, np.sort(lam), rtol=0, atol=1e-13 * np.max(np.abs(lam)))
    assert np.max(rs) < 1e-12 * np.max(np.abs(lam))
    c.close()


def test_chebyshev_filter_complex_matches_oracle():
    c, V, A, ap = _ctx(8.0, 4, 4)
    X = _cblock(c.n_dof, 40, 9)
    b = c.upper_bound_k
    a, a0 = 2.0, -1.5
    Xg = _gpu(X)
    c.chebyshev_filter_complex(Xg, 15, a, b, a0, block_width=16)    # three blocks, the last ragged
    Zo = och.cheb_filter_scaled(ap, X, 15, a, b, a0)
    rel = np.max(np.abs(_host(Xg) - Zo)) / np.max(np.abs(Zo))
    assert rel < 1e-11, rel
    c.close()


def test_solve_complex_matches_dense_hermitian_eigensolve():
    L, n_el, p = 8.0, 4, 3
    c, V, A, ap = _ctx(L, n_el, p)
    ev, evec = np.linalg.eigh(kpoint.htilde_k_csr(L, n_el, p, V, K).toarray())
    N = 20
    nb = workload.block_size(N)
    X = _gpu(_cblock(c.n_dof, nb, 10))
    tol = 1e-9 * max(1.0, abs(ev[0]))
    out = c.solve_complex(X, N, 20, tol, max_iter=300)
    assert out["converged"], out
    err = np.abs(out["evals"][:N] - ev[:N]) / np.maximum(np.abs(ev[:N]), 1.0)
    assert np.max(err) < 1e-10, err
    Xs = _host(X)
    for k in och.cluster_boundaries(ev, N):
        Q1, _ = np.linalg.qr(Xs[:, :k])
        s = np.linalg.norm(evec[:, :k] - Q1 @ (Q1.conj().T @ evec[:, :k]), 2)
        assert np.arcsin(min(1.0, s)) < 1e-8, k
    r_true = np.linalg.norm(ap(Xs) - Xs * out["evals"][None, :], axis=0)
    np.testing.assert_allclose(out["resid"], r_true, rtol=1e-6, atol=1e-12)
    c.close()


def test_solve_complex_v_zero_gives_sums_of_1d_bloch_levels():
    L, n_el, p = 10.0, 6, 5
    c, V, A, ap = _ctx(L, n_el, p, wells=False)
    a = [np.linalg.eigvalsh(x) for x in A]
    sums = np.sort((a[2][:8, None, None] + a[1][None, :8, None] + a[0][None, None, :8]).reshape(-1))
    N = 24
    while sums[N] - sums[N - 1] < 1e-6:
        N += 1
    X = _gpu(_cblock(c.n_dof, workload.block_size(N), 11))
    out = c.solve_complex(X, N, 20, 1e-9, max_iter=300)
    assert out["converged"], out
    np.testing.assert_allclose(out["evals"][:N], sums[:N], rtol=1e-10, atol=1e-10)
    c.close()


def test_solve_complex_full_size_periodic_cell_sampled_columns():
    """The periodic cell with the 24^3-cell, degree-6 element size (2,985,984
    DoFs), k != 0, 32 states: two passes, then sampled Ritz pairs checked on
    the CPU through the oracle's Kronecker-sum operator (residuals, Rayleigh
    quotients) and the block's orthonormality."""
    import torch
    L, n_el, p = 40.0, 24, 6
    c, V, A, ap = _ctx(L, n_el, p, seed=2)
    nb = workload.block_size(32)
    g = torch.Generator(device="cuda:0").manual_seed(12)
    X = torch.randn((c.n_dof, nb), dtype=torch.complex128, device="cuda:0", generator=g)
    out = c.solve_complex(X, 32, 30, 1e-30, max_iter=2)
    assert out["iters"] == 2
    cols = [0, 5, 31, nb - 1]
    Xs = X[:, cols].cpu().numpy()
    G = Xs.conj().T @ Xs
    assert np.max(np.abs(G - np.eye(len(cols)))) < 1e-12
    lam = out["evals"][cols]
    HXs = ap(Xs)
    r_cpu = np.linalg.norm(HXs - Xs * lam[None, :], axis=0)
    np.testing.assert_allclose(out["resid"][cols], r_cpu, rtol=1e-7, atol=1e-11)
    rq = np.real(np.sum(Xs.conj() * HXs, axis=0))
    np.testing.assert_allclose(rq, lam, rtol=0, atol=1e-10 * max(1.0, np.max(np.abs(lam))))
    del X
    torch.cuda.empty_cache()
    c.close()
