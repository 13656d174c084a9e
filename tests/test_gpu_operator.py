"""GPU parity of the operator and the Chebyshev step against the oracle."""
import numpy as np
import pytest

from oracle import chfsi as och
from oracle import fem
import workload
from gpu_util import make_ctx, oracle_apply, tensor_eigvecs, to_gpu, to_host

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("n_el,p,ncols,ld", [
    (4, 4, 24, 24),      # small workload, one 64-column tile, partially used
    (4, 4, 1, 1),
    (3, 5, 65, 72),      # ragged second column tile, ld > ncols
    (2, 6, 130, 130),    # three tiles, last ragged
    (2, 7, 17, 20),      # p = 7 (two accumulator passes)
    (5, 3, 64, 64),
    (3, 2, 33, 40),
    (4, 1, 9, 9),
])
def test_apply_fp64_matches_oracle(n_el, p, ncols, ld):
    L = 2.5 * n_el
    wells = workload.draw_wells(4, L, 11 + p, (1.0, 3.0), (0.3, 0.6))
    c, V = make_ctx(L, n_el, p, wells=wells)
    X = workload.start_block(c.n_dof, ncols, 1000 + p)
    Xg = to_gpu(X, ld)
    Yg = c.apply(Xg)
    Y = to_host(Yg)
    Yo = oracle_apply(L, n_el, p, V)(X)
    assert _rel(Y, Yo) < 1e-13, _rel(Y, Yo)
    c.close()


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n_el,p,ncols", [(4, 4, 70), (3, 5, 65), (2, 6, 33), (2, 7, 20), (5, 3, 64), (3, 2, 40)])
def test_apply_tile_variants_match_oracle(variant, n_el, p, ncols):
    """Both cell-kernel tile configurations give the oracle's product (FP64 to
    rounding, FP32 at single-precision level)."""
    L = 2.5 * n_el
    wells = workload.draw_wells(4, L, 41 + p, (1.0, 3.0), (0.3, 0.6))
    c, V = make_ctx(L, n_el, p, wells=wells)
    c.set_tile_variant(variant)
    X = workload.start_block(c.n_dof, ncols, 3000 + p)
    Yo = oracle_apply(L, n_el, p, V)(X)
    e64 = _rel(to_host(c.apply(to_gpu(X))), Yo)
    e32 = _rel(to_host(c.apply(to_gpu(X), prec="fp32")), Yo)
    assert e64 < 1e-13, e64
    assert e32 < 2e-6, e32
    c.close()


def test_tile_variant_rejects_unknown():
    prob = workload.PROBLEMS["small"]
    c, _ = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    with pytest.raises(Exception):
        c.set_tile_variant(2)
    with pytest.raises(Exception):
        c.set_rr_residual(3)
    c.close()


def test_apply_fp32_close_to_oracle():
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block(c.n_dof, 40, 7)
    Y = to_host(c.apply(to_gpu(X), prec="fp32"))
    Yo = oracle_apply(prob.L, prob.n_el, prob.p, V)(X)
    assert _rel(Y, Yo) < 2e-6, _rel(Y, Yo)
    c.close()


def test_cheb_step_matches_formula():
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block(c.n_dof, 24, 8)
    Xp = workload.start_block(c.n_dof, 24, 9)
    Xg, Xpg = to_gpu(X), to_gpu(Xp)
    Yg = to_gpu(np.zeros_like(X))
    s1, s2, sh = 0.037, -0.81, 12.5
    c.cheb_step(Xg, Xpg, Yg, s1, s2, sh)
    ap = oracle_apply(prob.L, prob.n_el, prob.p, V)
    Yo = s1 * (ap(X) - sh * X) + s2 * Xp
    assert _rel(to_host(Yg), Yo) < 1e-13
    c.close()


def test_exact_eigenvectors_at_large_p6_shape():
    """Htilde x = lambda x for tensor-product eigenvectors (V = 0) at the
    24^3-cell, degree-6 shape (2,924,207 DoFs)."""
    prob = workload.PROBLEMS["large_p6"]
    X, lam, a = tensor_eigvecs(prob.L, prob.n_el, prob.p, [(0, 0, 0), (1, 2, 3), (7, 0, 5), (140, 141, 142)])
    c, _ = make_ctx(prob.L, prob.n_el, prob.p, V=np.zeros(prob.n_dof))
    Y = to_host(c.apply(to_gpu(X)))
    lam_max = 3 * a[-1]
    err = np.max(np.abs(Y - X * lam[None, :]))
    assert err < 1e-13 * lam_max, err
    c.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-4)])
def test_filter_scales_exact_eigenvectors(prec, tol):
    """Filter(x) = T_m(xi)/T_m(xi0) x for exact eigenvectors (eq. chebFilter)."""
    L, n_el, p = 12.0, 4, 5
    X, lam, a = tensor_eigvecs(L, n_el, p, [(0, 0, 0), (1, 0, 0), (2, 2, 1), (4, 3, 3), (9, 1, 0), (18, 18, 18)])
    c, _ = make_ctx(L, n_el, p, V=np.zeros((n_el * p - 1) ** 3))
    b = c.upper_bound
    a_lo, a0, m = lam[2] + 0.05, lam[0], 20
    Xg = to_gpu(X)
    c.chebyshev_filter(Xg, m, a_lo, b, a0, prec=prec, block_width=4)
    cc, e = 0.5 * (a_lo + b), 0.5 * (b - a_lo)
    scale = och.cheb_T(m, (lam - cc) / e) / och.cheb_T(m, np.array([(a0 - cc) / e]))[0]
    got = to_host(Xg)
    assert np.max(np.abs(got - X * scale[None, :])) < tol * np.max(np.abs(scale))
    c.close()


def test_filter_matches_oracle_small_workload():
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block(c.n_dof, prob.nblock, prob.x0_seed)
    b = c.upper_bound
    a, a0 = 1.5, -1.8
    Xg = to_gpu(X)
    c.chebyshev_filter(Xg, prob.degree, a, b, a0, block_width=16)  # two blocks, second ragged
    Zo = och.cheb_filter_scaled(oracle_apply(prob.L, prob.n_el, prob.p, V), X, prob.degree, a, b, a0)
    assert _rel(to_host(Xg), Zo) < 1e-11
    c.close()


@pytest.mark.parametrize("variant", [-1, 1])
@pytest.mark.parametrize("n_el,p,ncols", [(4, 4, 24), (3, 6, 70), (2, 7, 33), (4, 5, 64)])
def test_apply_bf16_and_split_accuracy(n_el, p, ncols, variant):
    """BF16 inputs with FP32 accumulation: error at the BF16 rounding level
    (2^-8 relative per operand); the hi/lo split recovers about 2^-16.
    Variant 1 runs the BF16 kernel on 32-column tiles."""
    L = 2.5 * n_el
    wells = workload.draw_wells(4, L, 31 + p, (1.0, 3.0), (0.3, 0.6))
    c, V = make_ctx(L, n_el, p, wells=wells)
    c.set_tile_variant(variant)
    X = workload.start_block(c.n_dof, ncols, 2000 + p)
    Yo = oracle_apply(L, n_el, p, V)(X)
    e_bf = _rel(to_host(c.apply(to_gpu(X), prec="bf16")), Yo)
    e_x3 = _rel(to_host(c.apply(to_gpu(X), prec="bf16x3")), Yo)
    e_32 = _rel(to_host(c.apply(to_gpu(X), prec="fp32")), Yo)
    assert e_bf < 3e-2, e_bf
    assert e_x3 < 2e-4, e_x3
    assert e_x3 < e_bf / 20
    assert e_32 < 2e-6
    c.close()


def test_filter_bf16_keeps_wanted_subspace_small_workload():
    """One degree-20 BF16 filter pass followed by FP64 CholGS + RR moves the
    Ritz values of the wanted states close to the FP64 filter's."""
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block(c.n_dof, prob.nblock, prob.x0_seed)
    b = c.upper_bound
    evs = {}
    for prec in ["fp64", "bf16", "bf16x3"]:
        Xg = to_gpu(X)
        c.orthonormalize(Xg)
        ev0, _ = c.rayleigh_ritz(Xg)
        for _ in range(3):
            c.chebyshev_filter(Xg, prob.degree, ev0[-1], b, ev0[0], prec=prec)
            c.orthonormalize(Xg)
            ev0, _ = c.rayleigh_ritz(Xg)
        evs[prec] = ev0[:prob.nstates]
    assert np.max(np.abs(evs["bf16"] - evs["fp64"])) < 5e-2
    assert np.max(np.abs(evs["bf16x3"] - evs["fp64"])) < 1e-4
    c.close()


@pytest.mark.parametrize("n_el,p", [(4, 4), (3, 5), (2, 6)])
@pytest.mark.parametrize("cpt", [0, 1, 2, 4])
def test_cells_per_tile_settings_match_oracle(n_el, p, cpt):
    """Work-groups holding 1, 2 or 4 cells of a colour (16-, 32- or 64-column
    groups) compute the same products: FP64 and FP32 apply against the
    oracle for column counts that fill, straddle and under-fill the groups,
    and one filter step against the default setting bit for bit."""
    L = 2.5 * n_el
    wells = workload.draw_wells(4, L, 41 + p, (1.0, 3.0), (0.3, 0.6))
    c, V = make_ctx(L, n_el, p, wells=wells)
    c.set_cells_per_tile(cpt)
    ap = oracle_apply(L, n_el, p, V)
    for ncols in (8, 24, 40, 65, 128):
        X = workload.start_block(c.n_dof, ncols, 3000 + ncols)
        Yo = ap(X)
        assert _rel(to_host(c.apply(to_gpu(X))), Yo) < 1e-13
        assert _rel(to_host(c.apply(to_gpu(X), prec="fp32")), Yo) < 2e-6
    X = workload.start_block(c.n_dof, 40, 3100)
    b = c.upper_bound
    A = to_gpu(X)
    c.chebyshev_filter(A, 3, 0.5 * b, b, -1.0)
    c.set_cells_per_tile(1)
    B = to_gpu(X)
    c.chebyshev_filter(B, 3, 0.5 * b, b, -1.0)
    np.testing.assert_array_equal(to_host(A), to_host(B))
    c.close()


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7])
def test_single_cell_mesh(p):
    """One cell (n_el = 1: colour 0 holds the only cell, colours 1..7 are
    empty launches) with (p - 1)^3 interior DoFs: the product against the
    oracle in FP64, FP32 and BF16, and at p = 4 the full solve against the dense
    eigensolve."""
    L = 3.0
    c, V = make_ctx(L, 1, p, wells=workload.draw_wells(1, L, 70 + p, (1.0, 2.0), (0.4, 0.5)))
    ncols = 5
    X = workload.start_block(c.n_dof, ncols, 70 + p)
    Yo = oracle_apply(L, 1, p, V)(X)
    assert _rel(to_host(c.apply(to_gpu(X))), Yo) < 1e-13
    # reduced formats per output against (k u + n_loc u32) (|H||x|): the kinetic
    # and potential parts cancel in part, so a relative max-norm would not bound them
    HabsX = fem.apply_kron(np.abs(fem.operator_1d(L, 1, p)), np.abs(V), np.abs(X))
    n_loc = (p + 1) ** 3
    for prec, u in (("fp32", 2.0 ** -24), ("bf16", 2.0 ** -8), ("bf16x3", 2.0 ** -16)):
        err = np.abs(to_host(c.apply(to_gpu(X), prec=prec)) - Yo)
        assert np.all(err <= (3.0 * u + n_loc * 2.0 ** -24) * HabsX), prec
    if p == 4:
        ev = np.linalg.eigvalsh(fem.htilde_csr(L, 1, p, V).toarray())
        Xs = to_gpu(workload.start_block(c.n_dof, 8, 7))
        out = c.solve(Xs, 4, 10, 1e-10, max_iter=200)
        assert out["converged"], out
        np.testing.assert_allclose(out["evals"][:4], ev[:4], rtol=0, atol=1e-10 * max(1.0, abs(ev[0])))
    c.close()


def test_empty_and_malformed_blocks_are_rejected():
    """ncols < 1, ld < ncols and null pointers return CHFSI_ERR_ARG before any
    launch; the context stays usable."""
    import ctypes
    import torch
    prob = workload.PROBLEMS["small"]
    c, V = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = torch.zeros((c.n_dof, 4), dtype=torch.float64, device="cuda:0")
    Y = torch.zeros_like(X)
    px, py = ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr())
    assert c._lib.chfsi_apply(c._h, px, py, 4, 0, 0) == -1          # ncols = 0
    assert c._lib.chfsi_apply(c._h, px, py, 3, 4, 0) == -1          # ld < ncols
    assert c._lib.chfsi_apply(c._h, None, py, 4, 4, 0) == -1        # null input
    Xr = workload.start_block(c.n_dof, 4, 3)
    assert _rel(to_host(c.apply(to_gpu(Xr))), oracle_apply(prob.L, prob.n_el, prob.p, V)(Xr)) < 1e-13
    c.close()
