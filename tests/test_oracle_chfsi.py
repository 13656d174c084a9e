"""Pins of the oracle's ChFSI steps (CPU only)."""
import numpy as np
import pytest

from oracle import chfsi, fem
import workload


def _box(L=9.0, n_el=3, p=4, V=None):
    A = fem.operator_1d(L, n_el, p)
    n = A.shape[0]
    if V is None:
        V = np.zeros(n ** 3)
    return A, V, (lambda X: fem.apply_kron(A, V, X))


def _tensor_eigvecs(A, picks):
    a, U = np.linalg.eigh(A)
    cols, lams = [], []
    for (i, j, k) in picks:
        cols.append(np.kron(U[:, k], np.kron(U[:, j], U[:, i])))
        lams.append(a[i] + a[j] + a[k])
    return np.stack(cols, axis=1), np.array(lams)


def test_cheb_T_closed_form_matches_recurrence():
    x = np.linspace(-3, 3, 61)
    t0, t1 = np.ones_like(x), x.copy()
    for m in range(2, 12):
        t0, t1 = t1, 2 * x * t1 - t0
        np.testing.assert_allclose(chfsi.cheb_T(m, x), t1, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m", [1, 2, 7, 20, 30])
def test_filter_scales_exact_eigenvectors(m):
    """T_m(Hbar) x = T_m((lambda - c)/e) x for an eigenvector x (eq. chebFilter)."""
    A, V, apply = _box()
    X, lam = _tensor_eigvecs(A, [(0, 0, 0), (1, 0, 0), (2, 1, 0), (3, 3, 2), (9, 8, 7), (10, 10, 10)])
    b = fem.upper_bound(A, V)
    a, a0 = lam[2] + 0.3, lam[0]
    c, e = 0.5 * (a + b), 0.5 * (b - a)
    Y = chfsi.cheb_filter_paper(apply, X, m, a, b)
    want = chfsi.cheb_T(m, (lam - c) / e)
    np.testing.assert_allclose(Y, X * want[None, :], rtol=1e-11, atol=1e-12 * np.max(np.abs(want)))
    Z = chfsi.cheb_filter_scaled(apply, X, m, a, b, a0)
    want_s = want / chfsi.cheb_T(m, np.array([(a0 - c) / e]))[0]
    np.testing.assert_allclose(Z, X * want_s[None, :], rtol=1e-11, atol=1e-13)


def test_scaled_filter_equals_paper_filter_over_T_m():
    prob = workload.PROBLEMS["small"]
    A = fem.operator_1d(prob.L, prob.n_el, prob.p)
    V = workload.eval_wells(workload.problem_wells(prob), fem.dof_coords(prob.L, prob.n_el, prob.p))
    apply = lambda X: fem.apply_kron(A, V, X)
    X = workload.start_block(prob.n_dof, 8, 5)
    b = fem.upper_bound(A, V)
    a, a0 = 2.0, -1.5
    m = 20
    c, e = 0.5 * (a + b), 0.5 * (b - a)
    Y = chfsi.cheb_filter_paper(apply, X, m, a, b)
    Z = chfsi.cheb_filter_scaled(apply, X, m, a, b, a0)
    tm = chfsi.cheb_T(m, np.array([(a0 - c) / e]))[0]
    np.testing.assert_allclose(Z, Y / tm, rtol=1e-9, atol=1e-12 * np.max(np.abs(Y / tm)))


def test_filter_coefficients_reproduce_scaled_filter():
    A, V, apply = _box(n_el=2, p=3)
    X = np.random.default_rng(3).standard_normal((A.shape[0] ** 3, 4))
    a, b, a0 = 1.0, fem.upper_bound(A, V), 0.2
    z_prev, z = None, X.copy()
    for (s1, s2, sh) in chfsi.filter_coefficients(9, a, b, a0):
        y = s1 * (apply(z) - sh * z) + (s2 * z_prev if z_prev is not None else 0.0)
        z_prev, z = z, y
    np.testing.assert_allclose(z, chfsi.cheb_filter_scaled(apply, X, 9, a, b, a0), rtol=1e-12, atol=1e-14)


def test_cholgs_matches_householder_qr():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((500, 24)) @ np.diag(np.logspace(0, 3, 24))
    Xo = chfsi.cholgs(X)
    Q, R = np.linalg.qr(X)
    Q = Q * np.sign(np.diag(R))[None, :]
    kappa = np.linalg.cond(X)
    assert np.max(np.abs(Xo - Q)) < 1e-13 * kappa ** 2
    assert np.max(np.abs(Xo.T @ Xo - np.eye(24))) < 1e-13 * kappa ** 2


def test_cholgs_rank_deficient_raises():
    rng = np.random.default_rng(12)
    X = rng.standard_normal((200, 6))
    X[:, 4] = X[:, 1]
    with pytest.raises(chfsi.NotSPD):
        chfsi.cholgs(X)


def test_cholgs_mixed_is_fp32_accurate_and_exact_on_diagonal_blocks():
    """Mixed CholGS: X^T X = I to FP32 level, and with bv >= ncols it reduces
    to the FP64 routine exactly (its steps are pinned in test_oracle_mixed)."""
    rng = np.random.default_rng(13)
    X = rng.standard_normal((2000, 40))
    Xm = chfsi.cholgs_mixed(X, bv=8)
    assert np.max(np.abs(Xm.T @ Xm - np.eye(40))) < 1e-5
    np.testing.assert_allclose(chfsi.cholgs_mixed(X, bv=64), chfsi.cholgs(X), rtol=0, atol=1e-14)


def test_rr_recovers_exact_pairs_from_rotated_eigenvectors():
    A, V, apply = _box()
    picks = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (2, 0, 0), (3, 1, 1), (2, 2, 2)]
    X, lam = _tensor_eigvecs(A, picks)
    Qr, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((len(picks), len(picks))))
    Xr, HXr, D, res = chfsi.rayleigh_ritz(apply, X @ Qr)
    np.testing.assert_allclose(D, np.sort(lam), rtol=1e-13, atol=1e-13)
    assert np.max(res) < 1e-12 * np.max(np.abs(lam))
    np.testing.assert_allclose(HXr, apply(Xr), atol=1e-12 * np.max(np.abs(lam)))


def test_solve_small_workload_matches_dense_eigh():
    prob = workload.PROBLEMS["small"]
    xyz = fem.dof_coords(prob.L, prob.n_el, prob.p)
    V = workload.eval_wells(workload.problem_wells(prob), xyz)
    H = fem.htilde_csr(prob.L, prob.n_el, prob.p, V)
    ev, evec = chfsi.eig_dense(H)
    A = fem.operator_1d(prob.L, prob.n_el, prob.p)
    apply = lambda X: fem.apply_kron(A, V, X)
    X0 = workload.start_block(prob.n_dof, prob.nblock, prob.x0_seed)
    tol = 1e-9 * max(1.0, abs(ev[0]))
    out = chfsi.chfsi_solve(apply, X0, prob.nstates, prob.degree, fem.upper_bound(A, V), tol)
    assert out["converged"]
    N = prob.nstates
    err = np.abs(out["evals"][:N] - ev[:N]) / np.maximum(np.abs(ev[:N]), 1.0)
    assert np.max(err) < 1e-10
    for k in chfsi.cluster_boundaries(ev, N):
        assert chfsi.subspace_angle(out["evecs"][:, :k], evec[:, :k]) < 1e-8


def test_dense_and_lanczos_agree_on_small_workload():
    prob = workload.PROBLEMS["small"]
    xyz = fem.dof_coords(prob.L, prob.n_el, prob.p)
    V = workload.eval_wells(workload.problem_wells(prob), xyz)
    H = fem.htilde_csr(prob.L, prob.n_el, prob.p, V)
    ev, _ = chfsi.eig_dense(H)
    A = fem.operator_1d(prob.L, prob.n_el, prob.p)
    w, _ = chfsi.eig_lanczos(lambda v: fem.apply_kron(A, V, v), prob.n_dof, 20)
    np.testing.assert_allclose(w, ev[:20], rtol=1e-12, atol=1e-12)


def test_subspace_angle_closed_form_and_library():
    """Two lines in the plane at angle theta (closed form), and random
    subspaces against scipy's principal angles; tiny angles stay resolved."""
    import scipy.linalg as sla
    for th in (0.0, 1e-12, 1e-6, 0.3, 1.2):
        a = np.array([[1.0], [0.0]])
        b = np.array([[np.cos(th)], [np.sin(th)]])
        assert abs(chfsi.subspace_angle(a, b) - th) < 1e-15 + 1e-12 * th
    rng = np.random.default_rng(7)
    for k in (1, 3, 8):
        A = rng.standard_normal((40, k))
        B = rng.standard_normal((40, k))
        want = np.max(sla.subspace_angles(A, B))
        assert abs(chfsi.subspace_angle(A, B) - want) < 1e-12
    # the same span in another basis
    A = np.linalg.qr(rng.standard_normal((30, 5)))[0]
    assert chfsi.subspace_angle(A, A @ np.linalg.qr(rng.standard_normal((5, 5)))[0]) < 1e-14


def test_cluster_boundaries_by_construction():
    ev = np.array([-1.0, -0.9995, -0.5, -0.5, -0.49995, 0.2, 0.7])
    # gaps of at least 1e-3 close the first 2, 5 and 6 values (-0.9995 -> -0.5,
    # -0.49995 -> 0.2, 0.2 -> 0.7); the others are 5e-4, 0 and 5e-5
    assert chfsi.cluster_boundaries(ev, 6) == [2, 5, 6]
    assert chfsi.cluster_boundaries(ev, 3) == [2]
    assert chfsi.cluster_boundaries(ev, 10) == [2, 5, 6]    # capped at the last index
    assert chfsi.cluster_boundaries(ev, 6, gap=0.6) == [5]       # only the 0.69995 gap
    assert chfsi.cluster_boundaries(ev, 6, gap=0.7) == []
