"""The allocation-free CholGS (chfsi_orthonormalize_noalloc) against the
allocating entry point, through the C ABI: two calls in a row, the second
with a smaller block, and a block large enough that the overlap runs with
fewer row splits than the allocating path."""
import ctypes as C

import numpy as np
import pytest

import workload
from gpu_util import make_ctx, to_gpu, to_host

pytestmark = pytest.mark.gpu


def _noalloc(c, X, mixed=0):
    px, ld, n = c._block(X)
    return c._lib.chfsi_orthonormalize_noalloc(c._h, px, ld, n, int(mixed))


def _compare(c, X, ld=None, mixed=0):
    A = to_gpu(X, ld)
    B = to_gpu(X, ld)
    c.orthonormalize(A, mixed=bool(mixed))
    st = _noalloc(c, B, mixed)
    assert st == 0, (st, c._lib.chfsi_last_error(c._h))
    a, b = to_host(A), to_host(B)
    kappa = np.linalg.cond(X)
    tol = (1e-13 if not mixed else 4e-7) * kappa ** 2
    assert np.max(np.abs(a - b)) < tol, np.max(np.abs(a - b))
    if not mixed:
        Q, R = np.linalg.qr(X)
        Q = Q * np.sign(np.diag(R))[None, :]
        assert np.max(np.abs(b - Q)) < 1e-13 * kappa ** 2
    assert np.max(np.abs(b.T @ b - np.eye(X.shape[1]))) < (1e-12 if not mixed else 1e-5)


def test_noalloc_cholgs_matches_the_allocating_entry_point_twice():
    prob = workload.PROBLEMS["small"]
    c, _ = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X1 = workload.start_block(c.n_dof, 200, 71) @ np.diag(np.logspace(0, 2, 200))
    _compare(c, X1)
    X2 = workload.start_block(c.n_dof, 40, 72)        # second call, smaller, another row stride
    _compare(c, X2, ld=48)
    _compare(c, X2, mixed=1)
    c.close()


def test_noalloc_cholgs_with_capped_overlap_splits():
    """262,144 rows x 256 columns: the allocating overlap uses more row splits
    than the static array's partial region holds, so this path runs fewer."""
    L, n_el, p = 26.0, 13, 5
    wells = workload.draw_wells(8, L, 21, (1.0, 3.0), (0.5, 1.5))
    c, _ = make_ctx(L, n_el, p, wells=wells)
    X = workload.start_block(c.n_dof, 256, 73)
    _compare(c, X)
    _compare(c, workload.start_block(c.n_dof, 130, 74))
    c.close()


def test_noalloc_rejects_blocks_above_the_limit_and_leaves_them_untouched():
    prob = workload.PROBLEMS["small"]
    c, _ = make_ctx(prob.L, prob.n_el, prob.p, wells=workload.problem_wells(prob))
    X = workload.start_block(c.n_dof, 257, 75)
    Xg = to_gpu(X)
    assert _noalloc(c, Xg) == -1
    assert b"limit" in c._lib.chfsi_last_error(c._h)
    np.testing.assert_array_equal(to_host(Xg), X)
    Xr = workload.start_block(c.n_dof, 24, 76)
    Xr[:, 5] = Xr[:, 2]
    Xg = to_gpu(Xr)
    assert _noalloc(c, Xg) == -5                       # rank deficient: NOT_SPD, X unchanged
    np.testing.assert_array_equal(to_host(Xg), Xr)
    c.close()
