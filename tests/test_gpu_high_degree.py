"""GPU parity of the row-group cell kernel for GLL degrees 8..12 (n_loc =
729..2197 local nodes, cell matrices of 4.2..38.6 MB in FP64) against the
oracle's Kronecker-sum operator, and a full solve against dense eigh."""
import numpy as np
import pytest

from oracle import chfsi as och
from oracle import fem
import workload
from gpu_util import make_ctx, oracle_apply, to_gpu, to_host

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("n_el,p", [(1, 8), (2, 8), (2, 9), (1, 10), (2, 11), (1, 12), (2, 12)])
def test_apply_high_degree_matches_oracle(n_el, p):
    L = 5.0 * n_el
    wells = workload.draw_wells(3, L, 60 + p, (1.0, 3.0), (0.3, 0.6))
    c, V = make_ctx(L, n_el, p, wells=wells)
    ap = oracle_apply(L, n_el, p, V)
    for ncols in (1, 37, 64, 130):
        X = workload.start_block(c.n_dof, ncols, 700 + ncols)
        Yo = ap(X)
        assert _rel(to_host(c.apply(to_gpu(X))), Yo) < 1e-13
        assert _rel(to_host(c.apply(to_gpu(X), prec="fp32")), Yo) < 5e-6
    c.close()


def test_bf16_is_refused_above_p7():
    import paper_1903_10959_amd as P
    c, _ = make_ctx(5.0, 2, 8)
    X = to_gpu(workload.start_block(c.n_dof, 8, 1))
    with pytest.raises(P.ChfsiError) as ei:
        c.apply(X, prec="bf16")
    assert ei.value.status == -1
    c.close()


def test_filter_and_solve_at_p8_match_oracle():
    prob_L, n_el, p = 6.0, 2, 8
    wells = workload.draw_wells(3, prob_L, 77, (1.0, 3.0), (0.4, 0.8))
    c, V = make_ctx(prob_L, n_el, p, wells=wells)
    ap = oracle_apply(prob_L, n_el, p, V)
    X = workload.start_block(c.n_dof, 24, 78)
    b = c.upper_bound
    Xg = to_gpu(X)
    c.chebyshev_filter(Xg, 12, 0.3 * b, b, -2.0, block_width=16)
    Zo = och.cheb_filter_scaled(ap, X, 12, 0.3 * b, b, -2.0)
    assert _rel(to_host(Xg), Zo) < 1e-11
    ev = np.linalg.eigvalsh(fem.htilde_csr(prob_L, n_el, p, V).toarray())
    N = 12
    Xs = to_gpu(workload.start_block(c.n_dof, workload.block_size(N), 79))
    out = c.solve(Xs, N, 20, 1e-9 * max(1.0, abs(ev[0])), max_iter=300)
    assert out["converged"], out
    err = np.abs(out["evals"][:N] - ev[:N]) / np.maximum(np.abs(ev[:N]), 1.0)
    assert np.max(err) < 1e-10, err
    c.close()
