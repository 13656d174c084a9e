"""The seeded input recipe (CPU only): the workloads' sizes as the
configurations state them, the guard-state rule, and the Gaussian-well
potential's definition."""
import numpy as np
import pytest

import workload


@pytest.mark.parametrize("name,n_dof,n_cells,n_loc,nstates,nblock,degree,width", [
    ("small", 3375, 64, 125, 16, 24, 20, 24),
    ("large_p6", 2924207, 13824, 343, 512, 568, 30, 128),
    ("large_p5", 4019679, 32768, 216, 1024, 1128, 30, 128),
])
def test_workload_sizes(name, n_dof, n_cells, n_loc, nstates, nblock, degree, width):
    prob = workload.PROBLEMS[name]
    assert prob.n_dof == n_dof == (prob.n_el * prob.p - 1) ** 3
    assert prob.n_el ** 3 == n_cells and (prob.p + 1) ** 3 == n_loc
    assert (prob.nstates, prob.nblock, prob.degree) == (nstates, nblock, degree)
    assert min(prob.block_width, prob.nblock) == width


def test_guard_state_rule():
    for n, nb in [(1, 8), (16, 24), (40, 48), (256, 288), (512, 568), (1024, 1128)]:
        assert workload.block_size(n) == nb
    for n in range(1, 600):
        nb = workload.block_size(n)
        assert nb % 8 == 0 and nb - n >= max(4, -(-n // 10)) and nb - n < max(4, -(-n // 10)) + 8


def test_wells_drawn_inside_the_box_within_their_ranges():
    w = workload.draw_wells(64, 40.0, 102, (1.0, 3.0), (0.5, 1.5))
    assert w.centres.shape == (64, 3)
    assert np.all(w.centres >= 4.5) and np.all(w.centres <= 40.0 - 4.5)
    assert np.all((w.depths >= 1.0) & (w.depths <= 3.0))
    assert np.all((w.widths >= 0.5) & (w.widths <= 1.5))
    # seeded: the same draw twice
    w2 = workload.draw_wells(64, 40.0, 102, (1.0, 3.0), (0.5, 1.5))
    np.testing.assert_array_equal(w.centres, w2.centres)


def test_well_potential_definition():
    """One well: -d at its centre, -d e^{-1/2} one width away (a standard
    deviation), and the sum of wells is additive; chunking changes nothing."""
    one = workload.Wells(np.array([[1.0, 2.0, 3.0]]), np.array([2.5]), np.array([0.7]))
    pts = np.array([[1.0, 2.0, 3.0], [1.7, 2.0, 3.0], [1.0, 2.0, 2.3]])
    v = workload.eval_wells(one, pts)
    np.testing.assert_allclose(v, [-2.5, -2.5 * np.exp(-0.5), -2.5 * np.exp(-0.5)], rtol=1e-15)
    two = workload.Wells(np.array([[1.0, 2.0, 3.0], [4.0, 4.0, 4.0]]), np.array([2.5, 1.0]), np.array([0.7, 1.2]))
    other = workload.Wells(two.centres[1:], two.depths[1:], two.widths[1:])
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 6, size=(1000, 3))
    np.testing.assert_allclose(workload.eval_wells(two, x),
                               workload.eval_wells(one, x) + workload.eval_wells(other, x), rtol=1e-14)
    np.testing.assert_array_equal(workload.eval_wells(two, x, chunk=7), workload.eval_wells(two, x))
