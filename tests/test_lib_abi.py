"""The C-ABI library on the CPU: exported symbols, host tables against the
oracle (bit-exact integer maps), bound and footprint -- no device calls."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import fem
import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chfsi.h")


def _lib_or_skip():
    import paper_1903_10959_amd as P
    if not os.path.exists(P.library_path()):
        pytest.skip("libchfsi.so not built (run __graft_entry__.build())")
    return P


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chfsi_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_paper_operations():
    syms = declared_symbols()
    for s in ["chfsi_set_mesh", "chfsi_set_potential", "chfsi_chebyshev_filter", "chfsi_orthonormalize",
              "chfsi_rayleigh_ritz", "chfsi_solve", "chfsi_apply", "chfsi_create", "chfsi_destroy"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    P = _lib_or_skip()
    lib = ctypes.CDLL(P.library_path())
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1903_10959_amd import _lib
    assert set(declared_symbols()) <= set(_lib.SIGNATURES)


@pytest.mark.parametrize("L,n_el,p", [(10.0, 4, 4), (7.5, 3, 5), (5.0, 2, 7), (9.0, 5, 6), (3.0, 1, 2), (4.0, 2, 1)])
def test_host_tables_match_oracle(L, n_el, p):
    P = _lib_or_skip()
    c = P.Context(device=-1).set_mesh(L, n_el, p)
    assert c.n_dof == (n_el * p - 1) ** 3 and c.n_cells == n_el ** 3 and c.n_loc == (p + 1) ** 3
    # integer tables: bit-exact
    np.testing.assert_array_equal(c.cell_dof_map(), fem.cell_dof_map(n_el, p))
    np.testing.assert_array_equal(c.cell_colors(), fem.cell_colors(n_el))
    # floating-point tables: independent implementations, agree to rounding
    K, M = fem.assemble(L, n_el, p)
    np.testing.assert_allclose(c.mass(), M, rtol=1e-14)
    Ke = fem.cell_stiffness(p, L / n_el)
    assert np.max(np.abs(c.cell_matrix() - Ke)) < 1e-13 * np.max(np.abs(Ke))
    np.testing.assert_allclose(c.dof_coords(), fem.dof_coords(L, n_el, p), rtol=0, atol=1e-13 * L)
    c.close()


def test_upper_bound_host_only():
    P = _lib_or_skip()
    prob = workload.PROBLEMS["small"]
    c = P.Context(device=-1).set_mesh(prob.L, prob.n_el, prob.p)
    V = workload.eval_wells(workload.problem_wells(prob), c.dof_coords())
    c.set_potential(V)
    A = fem.operator_1d(prob.L, prob.n_el, prob.p)
    b_oracle = fem.upper_bound(A, V)
    lmax = np.linalg.eigvalsh(fem.htilde_csr(prob.L, prob.n_el, prob.p, V).toarray())[-1]
    assert c.upper_bound >= lmax
    assert abs(c.upper_bound - b_oracle) < 1e-10 * b_oracle


def test_host_only_context_refuses_device_work():
    P = _lib_or_skip()
    c = P.Context(device=-1).set_mesh(10.0, 2, 3)
    st = c._lib.chfsi_apply(c._h, ctypes.c_void_p(16), ctypes.c_void_p(32), 4, 4, 0)
    assert st == -2  # CHFSI_ERR_STATE
    assert b"host-only" in c._lib.chfsi_last_error(c._h)


def test_invalid_mesh_arguments_are_rejected():
    P = _lib_or_skip()
    c = P.Context(device=-1)
    for args in [(10.0, 0, 4), (-1.0, 2, 2), (10.0, 2, 13), (10.0, 1, 1)]:
        with pytest.raises(P.ChfsiError):
            c.set_mesh(*args)


def test_footprint_is_consistent():
    P = _lib_or_skip()
    small = P.footprint_bytes(4, 4, 24, 24)
    big = P.footprint_bytes(24, 6, 568, 128)
    assert 0 < small < big
    nd = (24 * 6 - 1) ** 3
    # at least X-sized HX workspace plus three filter buffers
    assert big >= nd * 568 * 8 + 3 * nd * 128 * 8
    assert P.footprint_bytes(24, 6, 568, 128, "fp32") < big


@pytest.mark.parametrize("p", [8, 12])
def test_high_degrees_build_and_have_fp64_footprints_only(p):
    """p = 8..12 build their tables (row-group cell kernel in FP64/FP32); the
    BF16 kernel and the batch session stop at p = 7, and p = 13 is refused."""
    P = _lib_or_skip()
    c = P.Context(device=-1).set_mesh(10.0, 2, p)
    assert c.n_loc == (p + 1) ** 3
    np.testing.assert_array_equal(c.cell_dof_map(), fem.cell_dof_map(2, p))
    c.close()
    assert P.footprint_bytes(2, p, 8) > 0 and P.footprint_bytes(2, p, 8, 0, "fp32") > 0
    assert P.footprint_bytes(2, p, 8, 0, "bf16") == 0 and P.batch_footprint_bytes(2, p, 8) == 0
    with pytest.raises(P.ChfsiError):
        P.Context(device=-1).set_mesh(10.0, 2, 13)


def test_batch_footprint_counts_every_session_buffer():
    """What a context holds in a batch session: at least its three FP64-sized
    recursion buffers, HX and the N_b x N_b matrices, and no less than the
    standalone-solve footprint with an FP32 filter of the same width."""
    P = _lib_or_skip()
    n_el, p, nb = 12, 7, 288
    nd = (n_el * p - 1) ** 3
    fb = P.batch_footprint_bytes(n_el, p, nb)
    assert fb >= 4 * nd * nb * 8 + 3 * nb * nb * 8
    assert fb >= P.footprint_bytes(n_el, p, nb, nb, "fp32")
    assert fb < 6 * nd * nb * 8
    assert P.batch_footprint_bytes(4, 4, 24) < fb
