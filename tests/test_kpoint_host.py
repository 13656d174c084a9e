"""Host tables of the periodic mesh against the oracle (integer maps
bit-exact), the periodic spectral bound, and argument checks; CPU only (a
host-only context touches no GPU)."""
import numpy as np
import pytest

import paper_1903_10959_amd as P
from oracle import fem, kpoint
import workload


@pytest.mark.parametrize("L,n_el,p", [(5.0, 2, 3), (8.0, 4, 4), (6.0, 2, 6), (4.0, 2, 1), (9.0, 6, 2)])
def test_periodic_host_tables_match_oracle(L, n_el, p):
    c = P.Context(device=-1).set_mesh(L, n_el, p, periodic=True)
    assert c.n_dof == (n_el * p) ** 3 and c.n_cells == n_el ** 3
    np.testing.assert_array_equal(c.cell_dof_map(), kpoint.cell_dof_map_periodic(n_el, p))
    np.testing.assert_array_equal(c.cell_colors(), fem.cell_colors(n_el))
    _, _, M = kpoint.assemble_periodic(L, n_el, p)
    np.testing.assert_allclose(c.mass(), M, rtol=1e-14)
    np.testing.assert_allclose(c.dof_coords(), kpoint.dof_coords_periodic(L, n_el, p), rtol=0, atol=1e-13 * L)
    c.close()


def test_periodic_upper_bound_is_rigorous():
    L, n_el, p = 6.0, 2, 4
    c = P.Context(device=-1).set_mesh(L, n_el, p, periodic=True)
    V = workload.eval_wells(workload.draw_wells(3, L, 4, (1.0, 2.0), (0.5, 1.0)), c.dof_coords())
    c.set_potential(V)
    lmax = np.linalg.eigvalsh(kpoint.htilde_k_csr(L, n_el, p, V, [0, 0, 0]).toarray())[-1].real
    A1 = kpoint.operator_1d_periodic(L, n_el, p, 0.0).real
    b = 3 * np.linalg.eigvalsh(A1)[-1] + V.max()
    assert lmax <= c.upper_bound
    assert abs(c.upper_bound - b) < 1e-10 * b
    c.close()


def test_periodic_argument_checks():
    with pytest.raises(P.ChfsiError):
        P.Context(device=-1).set_mesh(5.0, 3, 3, periodic=True)       # odd n_el
    c = P.Context(device=-1).set_mesh(5.0, 2, 3)
    with pytest.raises(P.ChfsiError):
        c.set_kpoint((0.1, 0.0, 0.0))                               # not periodic
    c.close()
    c = P.Context(device=-1).set_mesh(5.0, 2, 3, periodic=True)
    c.set_kpoint((0.1, -0.2, 0.3))
    with pytest.raises(P.ChfsiError):
        c.set_kpoint((np.inf, 0.0, 0.0))
    c.close()


def test_kpoint_group_argument_checks():
    c = P.Context(device=-1).set_mesh(5.0, 2, 3)
    with pytest.raises(P.ChfsiError):
        c.set_kpoints([[0.1, 0.0, 0.0]])                            # not periodic
    c.close()
    c = P.Context(device=-1).set_mesh(5.0, 2, 3, periodic=True)
    c.set_kpoints([[0.1, 0.0, 0.0], [0.0, 0.2, 0.0]])
    with pytest.raises(P.ChfsiError):
        c.set_kpoints([[0.1, np.nan, 0.0]])
    c.close()
