"""The fused element-wise pass relies on a first-touch rule evaluated in the
cell kernel: local node (a,b,c) of cell (ex,ey,ez) writes Y when, in every
direction, the node is interior to the cell or the cell's parity bit is 0.
Checked here against the oracle's map and colouring: exactly one (cell, node)
pair per DoF is a first touch, and its cell has the smallest colour among the
cells containing that DoF (colours are launched in increasing order)."""
import numpy as np
import pytest

from oracle import fem


def first_touch(r, q, e, n_el):
    a, b, c = r % q, (r // q) % q, r // (q * q)
    ex, ey, ez = e % n_el, (e // n_el) % n_el, e // (n_el * n_el)
    fx = (0 < a < q - 1) or not (ex & 1)
    fy = (0 < b < q - 1) or not (ey & 1)
    fz = (0 < c < q - 1) or not (ez & 1)
    return fx and fy and fz


@pytest.mark.parametrize("n_el,p", [(1, 2), (2, 2), (3, 3), (4, 4), (5, 2), (2, 6)])
def test_first_touch_is_unique_and_in_the_first_colour(n_el, p):
    cmap = fem.cell_dof_map(n_el, p)
    col = fem.cell_colors(n_el)
    q = p + 1
    nd = (n_el * p - 1) ** 3
    firsts = np.zeros(nd, dtype=int)
    min_col = np.full(nd, 99)
    first_col = np.full(nd, -1)
    for e in range(cmap.shape[0]):
        for r in range(cmap.shape[1]):
            d = cmap[e, r]
            if d < 0:
                continue
            min_col[d] = min(min_col[d], col[e])
            if first_touch(r, q, e, n_el):
                firsts[d] += 1
                first_col[d] = col[e]
    assert np.all(firsts == 1)
    np.testing.assert_array_equal(first_col, min_col)
