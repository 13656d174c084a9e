"""GPU parity of CholGS, Rayleigh-Ritz and the full solve against the oracle."""
import numpy as np
import pytest

from oracle import chfsi as och
from oracle import density as ode
from oracle import fem
import workload
from gpu_util import make_ctx, oracle_apply, tensor_eigvecs, to_gpu, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ncols,ld,scale_decades", [(24, 24, 3), (40, 48, 2), (130, 130, 1), (200, 200, 1)])
def test_orthonormalize_matches_householder(ncols, ld, scale_decades):
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    rng = np.random.default_rng(ncols)
    X = rng.standard_normal((c.n_dof, ncols)) @ np.diag(np.logspace(0, scale_decades, ncols))
    Xg = to_gpu(X, ld)
    c.orthonormalize(Xg)
    Xo = to_host(Xg)
    Q, R = np.linalg.qr(X)
    Q = Q * np.sign(np.diag(R))[None, :]
    kappa = np.linalg.cond(X)
    assert np.max(np.abs(Xo - Q)) < 1e-13 * kappa ** 2
    assert np.max(np.abs(Xo.T @ Xo - np.eye(ncols))) < 1e-13 * kappa ** 2
    np.testing.assert_allclose(Xo, och.cholgs(X), rtol=0, atol=1e-13 * kappa ** 2)
    c.close()


def test_orthonormalize_mixed_matches_oracle_mixed():
    """Mixed CholGS (eq. overlapmixedprec, 64-wide FP64 diagonal blocks):
    element by element against the oracle's mixed CholGS within a bound
    derived from the FP32 unit roundoff, and measurably apart from the FP64
    result (so the FP32 blocks really ran)."""
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block(c.n_dof, 150, 77)
    Xg = to_gpu(X)
    c.orthonormalize(Xg, mixed=True)
    Xm = to_host(Xg)
    Xo = och.cholgs_mixed(X, 64)
    Xd = och.cholgs(X)
    u32 = 2.0 ** -24
    kappa = np.linalg.cond(X)
    # FP32 sums of n products carry ~sqrt(n) u32 relative error; CholGS
    # amplifies an overlap error by kappa^2
    tol = 8.0 * np.sqrt(c.n_dof) * u32 * kappa ** 2 * np.max(np.abs(Xd))
    assert np.max(np.abs(Xm - Xo)) < tol, (np.max(np.abs(Xm - Xo)), tol)
    assert np.max(np.abs(Xm - Xd)) > 1e-10, np.max(np.abs(Xm - Xd))
    assert np.max(np.abs(Xm.T @ Xm - np.eye(150))) < 5e-6
    c.close()


def test_orthonormalize_rank_deficient_reports_not_spd():
    import paper_1903_10959_amd as P
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block(c.n_dof, 24, 5)
    X[:, 7] = X[:, 3]
    Xg = to_gpu(X)
    with pytest.raises(P.ChfsiError) as ei:
        c.orthonormalize(Xg)
    assert ei.value.status == -5
    np.testing.assert_array_equal(to_host(Xg), X)     # X untouched on failure
    c.close()


def test_rayleigh_ritz_exact_on_rotated_eigenvectors():
    L, n_el, p = 9.0, 3, 4
    picks = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (2, 0, 0), (3, 1, 1), (2, 2, 2),
             (4, 0, 0), (0, 4, 1), (5, 5, 5), (10, 9, 8)]
    X, lam, _ = tensor_eigvecs(L, n_el, p, picks)
    Qr, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((len(picks), len(picks))))
    c, _ = make_ctx(L, n_el, p, V=np.zeros((n_el * p - 1) ** 3))
    Xg = to_gpu(X @ Qr)
    HX = to_gpu(np.zeros_like(X))
    ev, res = c.rayleigh_ritz(Xg, HX_out=HX)
    np.testing.assert_allclose(ev, np.sort(lam), rtol=1e-13, atol=1e-13)
    assert np.max(res) < 1e-12 * np.max(np.abs(lam))
    np.testing.assert_allclose(to_host(HX), oracle_apply(L, n_el, p, np.zeros(X.shape[0]))(to_host(Xg)),
                               atol=1e-12 * np.max(np.abs(lam)))
    c.close()


RR_COLS = [1, 2, 3, 24, 31, 32, 33, 63, 64, 65, 97, 129, 200]


@pytest.mark.parametrize("ncols,mode", [(n, 0) for n in RR_COLS] + [(n, m) for n in (1, 33, 129) for m in (1, 2)])
def test_rayleigh_ritz_matches_oracle(ncols, mode):
    """mode: how Htilde of the rotated columns is formed (0 cost model,
    1 rotating HX, 2 applying Htilde again); HX_out checked against the oracle."""
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    c.set_rr_residual(mode)
    X = och.cholgs(workload.start_block(c.n_dof, ncols, 300 + ncols))
    ap = oracle_apply(prob.L, prob.n_el, prob.p, V)
    Xr, HXr, D, res = och.rayleigh_ritz(ap, X)
    Xg = to_gpu(X)
    HX = to_gpu(np.zeros_like(X))
    ev, rs = c.rayleigh_ritz(Xg, HX_out=HX)
    scale = max(1.0, np.max(np.abs(D)))
    np.testing.assert_allclose(ev, D, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(rs, res, rtol=1e-6, atol=1e-11 * scale)
    assert np.max(np.abs(to_host(HX) - ap(to_host(Xg)))) < 1e-11 * scale
    # Ritz vectors up to sign (the projected spectrum of a random block is simple)
    G = to_host(Xg)
    sgn = np.sign(np.sum(G * Xr, axis=0))
    assert np.max(np.abs(G * sgn[None, :] - Xr)) < 1e-8
    c.close()


def test_solve_small_workload_matches_dense_eigh():
    """The plain definition: lowest 16 eigenpairs of Htilde by LAPACK."""
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    H = fem.htilde_csr(prob.L, prob.n_el, prob.p, V)
    ev, evec = och.eig_dense(H)
    X = to_gpu(workload.start_block(c.n_dof, prob.nblock, prob.x0_seed))
    N = prob.nstates
    tol = 1e-9 * max(1.0, abs(ev[0]))
    out = c.solve(X, N, prob.degree, tol, max_iter=200)
    assert out["converged"], out
    err = np.abs(out["evals"][:N] - ev[:N]) / np.maximum(np.abs(ev[:N]), 1.0)
    assert np.max(err) < 1e-10, err
    Xs = to_host(X)
    for k in och.cluster_boundaries(ev, N):
        assert och.subspace_angle(Xs[:, :k], evec[:, :k]) < 1e-8, k
    # every residual the library reports is the true residual of its vectors
    ap = oracle_apply(prob.L, prob.n_el, prob.p, V)
    r_true = np.linalg.norm(ap(Xs) - Xs * out["evals"][None, :], axis=0)
    np.testing.assert_allclose(out["resid"], r_true, rtol=1e-6, atol=1e-12)
    c.close()


def test_solve_box_closed_form_at_large_p6_shape_subset():
    """V = 0 on a mid-size mesh: lowest levels equal sums of 1D eigenvalues."""
    L, n_el, p = 20.0, 8, 6
    c, _ = make_ctx(L, n_el, p, V=np.zeros((n_el * p - 1) ** 3))
    a = np.linalg.eigvalsh(fem.operator_1d(L, n_el, p))
    sums = np.sort((a[:8, None, None] + a[None, :8, None] + a[None, None, :8]).reshape(-1))
    N = 20   # 1 + 3 + 3 + 3 + 6 + 4 ... stop at a cluster boundary
    while sums[N] - sums[N - 1] < 1e-6:
        N += 1
    nb = workload.block_size(N)
    X = to_gpu(workload.start_block(c.n_dof, nb, 55))
    out = c.solve(X, N, 20, 1e-9, max_iter=300)
    assert out["converged"]
    np.testing.assert_allclose(out["evals"][:N], sums[:N], rtol=1e-10, atol=1e-10)
    c.close()


def test_cholgs_and_rr_at_568_columns_across_row_chunks():
    """568 columns (the large_p6 block) on 262,144 DoFs: 1.49e8 elements, more
    than the rotation kernel's 2^27-element scratch panel holds, so the chunked
    path and its ragged last chunk are both exercised."""
    L, n_el, p = 26.0, 13, 5
    wells = workload.draw_wells(8, L, 21, (1.0, 3.0), (0.5, 1.5))
    c, V = make_ctx(L, n_el, p, wells=wells)
    X = workload.start_block(c.n_dof, 568, 31)
    Xg = to_gpu(X)
    c.orthonormalize(Xg)
    Xo = och.cholgs(X)
    kappa = np.linalg.cond(X)
    assert np.max(np.abs(to_host(Xg) - Xo)) < 1e-13 * kappa ** 2
    ev, rs = c.rayleigh_ritz(Xg)
    Xr, HXr, D, res = och.rayleigh_ritz(oracle_apply(L, n_el, p, V), Xo)
    scale = max(1.0, np.max(np.abs(D)))
    np.testing.assert_allclose(ev, D, rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(rs, res, rtol=1e-5, atol=1e-10 * scale)
    c.close()


@pytest.mark.parametrize("ladder,mixed", [(("bf16", "fp32", "fp64"), False), (("fp32", "fp64"), True)])
def test_solve_precision_ladder_reaches_fp64_accuracy(ladder, mixed):
    """Reduced-precision filter rungs, then FP64: the converged eigenvalues
    match dense eigh to the FP64 tolerance."""
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    ev = np.linalg.eigvalsh(fem.htilde_csr(prob.L, prob.n_el, prob.p, V).toarray())
    X = to_gpu(workload.start_block(c.n_dof, prob.nblock, prob.x0_seed))
    N = prob.nstates
    out = c.solve(X, N, prob.degree, 1e-9 * max(1.0, abs(ev[0])), max_iter=300, ladder=ladder,
                  mixed_cholgs=mixed)
    assert out["converged"]
    assert out["rung"] == len(ladder) - 1        # finished on the FP64 rung
    err = np.abs(out["evals"][:N] - ev[:N]) / np.maximum(np.abs(ev[:N]), 1.0)
    assert np.max(err) < (1e-10 if not mixed else 1e-8), err
    c.close()


@pytest.mark.parametrize("ncols,n_fr,mode", [(24, 4, 0), (97, 15, 0), (200, 30, 0), (200, 200, 0), (65, 1, 0),
                                             (97, 15, 1), (97, 15, 2), (200, 30, 1), (200, 30, 2)])
def test_rayleigh_ritz_split_fp64_equals_full(ncols, n_fr, mode):
    """Spectrum splitting with an all-FP64 projection: the N_fr largest Ritz
    pairs of the full Rayleigh-Ritz; the first N_oc columns untouched."""
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    c.set_rr_residual(mode)
    X = och.cholgs(workload.start_block(c.n_dof, ncols, 500 + ncols))
    ap = oracle_apply(prob.L, prob.n_el, prob.p, V)
    Xr, HXr, D, res = och.rayleigh_ritz(ap, X)
    n_oc = ncols - n_fr
    Xg = to_gpu(X)
    ev, rs = c.rayleigh_ritz_split(Xg, n_fr, mixed=False)
    scale = max(1.0, np.max(np.abs(D)))
    np.testing.assert_allclose(ev, D[n_oc:], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(rs, res[n_oc:], rtol=1e-6, atol=1e-11 * scale)
    G = to_host(Xg)
    assert np.array_equal(G[:, :n_oc], X[:, :n_oc])
    sgn = np.sign(np.sum(G[:, n_oc:] * Xr[:, n_oc:], axis=0))
    assert np.max(np.abs(G[:, n_oc:] * sgn[None, :] - Xr[:, n_oc:])) < 1e-8
    c.close()


def test_rayleigh_ritz_split_mixed_precision_accuracy():
    """Mixed projection (FP32 outside the fr-fr block, whose start the library
    rounds down to a multiple of 64): on a random block the N_fr largest Ritz
    values match the oracle's mixed split at the same block start within a
    few FP32 roundoffs of the spectrum's scale, and differ from the FP64
    values by far more than FP64 rounding; near convergence (the regime the
    paper's argument is made for) the coupling blocks vanish and the error
    drops far below it."""
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    ap = oracle_apply(prob.L, prob.n_el, prob.p, V)
    ncols, n_fr = 130, 20
    n_oc = ncols - n_fr
    fr0 = (n_oc // 64) * 64
    X = och.cholgs(workload.start_block(c.n_dof, ncols, 77))
    _, _, D, _ = och.rayleigh_ritz(ap, X)
    _, Dmix, _ = ode.rayleigh_ritz_split(ap, X, n_fr, mixed=True, fr0=fr0)
    ev, _ = c.rayleigh_ritz_split(to_gpu(X), n_fr, mixed=True)
    scale = np.max(np.abs(D))
    u32 = 2.0 ** -24
    np.testing.assert_allclose(ev, Dmix, rtol=0, atol=4.0 * u32 * scale)
    err_random = np.max(np.abs(ev - D[n_oc:]))
    assert 1e-9 < err_random < 1e-5 * scale, err_random
    # near-converged block: exact eigenvectors plus a 1e-4 perturbation
    H = fem.htilde_csr(prob.L, prob.n_el, prob.p, V)
    w, U = och.eig_dense(H)
    Xn = och.cholgs(U[:, :ncols] + 1e-4 * workload.start_block(c.n_dof, ncols, 78))
    _, _, Dn, _ = och.rayleigh_ritz(ap, Xn)
    evn, _ = c.rayleigh_ritz_split(to_gpu(Xn), n_fr, mixed=True)
    err_conv = np.max(np.abs(evn - Dn[n_oc:]))
    assert err_conv < 1e-8 * scale and err_conv < err_random / 10, (err_conv, err_random)
    c.close()
