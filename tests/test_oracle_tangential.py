"""Pin of the oracle's tangential differences (App. A.3.4, reading A10/A11): central
computational differences inside a block and one-sided ones next to a side without a
neighbour, for cell fields (Gt) and for Dirichlet values along a side (Bt).

Both forms are exact on fields linear in the cell index, so a linear field must give its
slope in every cell and on every face, next to walls and corners included; a one-sided
difference with a wrong weight (a half, or the central form with the missing neighbour
replaced by the cell itself) fails there (no GPU).
"""
import numpy as np
import pytest

import cases
from oracle.piso import Geometry


@pytest.mark.parametrize("make", [lambda: cases.lid_cavity(6, n_steps=1), lambda: cases.channel(4, 5, 3)])
def test_cell_differences_exact_on_linear_fields(make):
    case = make()
    geo = Geometry(case.domain)
    nx, ny, nz = case.domain.blocks[0]
    P = np.arange(geo.N)
    idx = [P % nx, (P // nx) % ny, P // (nx * ny)]
    # axes with walls on both ends (a linear field would jump across a periodic wrap)
    walls = [a for a in range(geo.d) if any(s.kind == "dirichlet" and s.side // 2 == a for s in case.domain.sides)]
    assert walls
    slopes = {a: 1.5 - a for a in walls}
    phi = sum(slopes[a] * idx[a] for a in walls) + 0.25
    for k in range(geo.d):
        g = geo.Gt[k] @ phi
        want = slopes.get(k, 0.0)
        assert np.max(np.abs(g - want)) <= 1e-12, (k, np.max(np.abs(g - want)))


def test_boundary_differences_exact_on_linear_values():
    case = cases.lid_cavity(7, n_steps=1)
    geo = Geometry(case.domain)
    nx = case.domain.blocks[0][0]
    ny = case.domain.blocks[0][1]
    i = geo.bP % nx
    j = (geo.bP // nx) % ny
    # along the faces of the y-sides the tangential index is i, along the x-sides it is j
    ub = np.where(geo.bj == 1, 2.0 * i - 1.0, -0.5 * j + 3.0)
    for k in range(geo.d):
        g = geo.Bt[k] @ ub
        on = geo.bj != k
        want = np.where(geo.bj == 1, 2.0, -0.5)
        assert np.max(np.abs(g[on] - want[on])) <= 1e-12
        assert np.all(g[~on] == 0.0)
