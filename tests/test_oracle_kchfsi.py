"""Pins of the oracle's complex (k-point) ChFSI steps (oracle/kchfsi.py):
Householder QR, exact Bloch eigenvectors, dense Hermitian eigensolves and
1D-sum spectra -- none of them uses the functions under test."""
import numpy as np
import pytest

from oracle import chfsi, kchfsi, kpoint
import workload

K = np.array([0.13, -0.21, 0.08])


def _ops(L, n_el, p, k=K):
    return [kpoint.operator_1d_periodic(L, n_el, p, kd) for kd in k]


def test_cholgs_c_equals_householder_qr_with_real_positive_r_diagonal():
    rng = np.random.default_rng(31)
    X = (rng.standard_normal((400, 24)) + 1j * rng.standard_normal((400, 24))) @ np.diag(np.logspace(0, 2, 24))
    Xo = kchfsi.cholgs_c(X)
    Q, R = np.linalg.qr(X)
    ph = np.diag(R) / np.abs(np.diag(R))
    Q = Q * ph[None, :]
    kappa = np.linalg.cond(X)
    assert np.max(np.abs(Xo - Q)) < 1e-13 * kappa ** 2
    assert np.max(np.abs(Xo.conj().T @ Xo - np.eye(24))) < 1e-13 * kappa ** 2
    # a real-only routine would fail here: the imaginary parts matter
    assert np.max(np.abs(Xo.imag)) > 0.1 * np.max(np.abs(Xo))


def test_cholgs_c_rank_deficient_raises():
    rng = np.random.default_rng(32)
    X = rng.standard_normal((100, 5)) + 1j * rng.standard_normal((100, 5))
    X[:, 3] = (0.3 - 0.7j) * X[:, 1]
    with pytest.raises(chfsi.NotSPD):
        kchfsi.cholgs_c(X)


def _bloch_eigvecs(L, n_el, p, picks, k=K):
    A = _ops(L, n_el, p, k)
    eig = [np.linalg.eigh(a) for a in A]
    cols, lam = [], []
    for (i, j, l) in picks:
        cols.append(np.kron(eig[2][1][:, l], np.kron(eig[1][1][:, j], eig[0][1][:, i])))
        lam.append(eig[0][0][i] + eig[1][0][j] + eig[2][0][l])
    return A, np.stack(cols, axis=1), np.array(lam)


def test_rayleigh_ritz_c_recovers_exact_bloch_pairs_from_a_unitary_mix():
    L, n_el, p = 6.0, 2, 4
    picks = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 1, 0), (3, 3, 3), (1, 2, 5), (4, 0, 2)]
    A, X, lam = _bloch_eigvecs(L, n_el, p, picks)
    V = np.zeros(X.shape[0])
    apply = lambda Y: kpoint.apply_kron_k(*A, V, Y)
    rng = np.random.default_rng(33)
    U, _ = np.linalg.qr(rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8)))
    Xr, HXr, D, res = kchfsi.rayleigh_ritz_c(apply, X @ U)
    np.testing.assert_allclose(D, np.sort(lam), rtol=0, atol=1e-13 * np.max(np.abs(lam)))
    assert np.max(res) < 1e-12 * np.max(np.abs(lam))
    np.testing.assert_allclose(HXr, apply(Xr), atol=1e-12 * np.max(np.abs(lam)))


def test_filter_on_exact_bloch_eigenvectors_scales_by_the_closed_form():
    L, n_el, p = 6.0, 2, 4
    picks = [(0, 0, 0), (2, 1, 0), (5, 5, 5), (7, 6, 7)]
    A, X, lam = _bloch_eigvecs(L, n_el, p, picks)
    V = np.zeros(X.shape[0])
    apply = lambda Y: kpoint.apply_kron_k(*A, V, Y)
    b = kchfsi.upper_bound_k(*A, V)
    a, a0, m = float(np.sort(lam)[1]) + 0.01, float(np.min(lam)) - 0.5, 12
    Z = chfsi.cheb_filter_scaled(apply, X, m, a, b, a0)
    c, e = 0.5 * (a + b), 0.5 * (b - a)
    scale = chfsi.cheb_T(m, (lam - c) / e) / chfsi.cheb_T(m, np.array([(a0 - c) / e]))[0]
    np.testing.assert_allclose(Z, X * scale[None, :], rtol=0, atol=1e-12 * np.max(np.abs(scale)))


def test_upper_bound_k_is_rigorous_and_tight():
    L, n_el, p = 6.0, 2, 3
    V = workload.eval_wells(workload.draw_wells(3, L, 7, (1.0, 3.0), (0.5, 1.0)), kpoint.dof_coords_periodic(L, n_el, p))
    lmax = np.linalg.eigvalsh(kpoint.htilde_k_csr(L, n_el, p, V, K).toarray())[-1]
    b = kchfsi.upper_bound_k(*_ops(L, n_el, p), V)
    assert lmax <= b <= 1.05 * lmax


def _solve_case(V_kind):
    L, n_el, p = 6.0, 2, 4
    xyz = kpoint.dof_coords_periodic(L, n_el, p)
    if V_kind == "wells":
        V = workload.eval_wells(workload.draw_wells(3, L, 8, (1.0, 3.0), (0.5, 1.0)), xyz)
    else:
        V = np.zeros(xyz.shape[0])
    A = _ops(L, n_el, p)
    apply = lambda Y: kpoint.apply_kron_k(*A, V, Y)
    rng = np.random.default_rng(34)
    n = xyz.shape[0]
    X0 = rng.standard_normal((n, 16)) + 1j * rng.standard_normal((n, 16))
    out = kchfsi.chfsi_solve_c(apply, X0, 12, 12, kchfsi.upper_bound_k(*A, V), 1e-9, max_iter=300)
    return L, n_el, p, V, A, out


def test_solve_c_matches_dense_hermitian_eigensolve():
    L, n_el, p, V, A, out = _solve_case("wells")
    assert out["converged"]
    ev, evec = np.linalg.eigh(kpoint.htilde_k_csr(L, n_el, p, V, K).toarray())
    N = 12
    err = np.abs(out["evals"][:N] - ev[:N]) / np.maximum(np.abs(ev[:N]), 1.0)
    assert np.max(err) < 1e-10, err
    for k in chfsi.cluster_boundaries(ev, N):
        Q1, _ = np.linalg.qr(out["evecs"][:, :k])
        Q2 = evec[:, :k]
        s = np.linalg.norm(Q2 - Q1 @ (Q1.conj().T @ Q2), 2)
        assert np.arcsin(min(1.0, s)) < 1e-8, k


def test_solve_c_at_v_zero_gives_sums_of_1d_bloch_levels():
    L, n_el, p, V, A, out = _solve_case("zero")
    assert out["converged"]
    a = [np.linalg.eigvalsh(x) for x in A]
    sums = np.sort((a[2][:, None, None] + a[1][None, :, None] + a[0][None, None, :]).reshape(-1))
    np.testing.assert_allclose(out["evals"][:12], sums[:12], rtol=1e-10, atol=1e-10)
