"""Pin of the boundary rows of the oracle's pressure gradient (reading A7: a boundary face
takes p_b = p_P, so the boundary cell's central difference becomes (p_+ - p_P) / 2).

With that reading the discrete gradient is minus the adjoint of the discrete divergence
of face-interpolated fluxes with no boundary flux (summation by parts):

    p . div(lerp(J T h)) = - sum_i sum_P J_P h_i,P (G_i p)_P

for every p and h, on any grid, interior, block connections and walls alike.  Another
boundary value (p_b = 0, a one-sided difference, a reflected ghost) breaks the identity
in the boundary rows, which is what the pin checks (no GPU).
"""
import numpy as np
import pytest

import cases
from oracle.piso import Geometry
from tests.test_oracle_pins import _two_block

GEOMS = [lambda: cases.lid_cavity(7, n_steps=1), lambda: cases.channel(4, 5, 3), _two_block,
         lambda: cases.sheared_channel(5, 6, shear=0.8), lambda: cases.cylinder_oh(8, 4, 3)]


@pytest.mark.parametrize("idx", range(len(GEOMS)))
def test_gradient_is_minus_adjoint_of_divergence(idx):
    geo = Geometry(GEOMS[idx]().domain)
    rng = np.random.default_rng(idx)
    p = rng.standard_normal(geo.N)
    h = rng.standard_normal((geo.d, geo.N))
    W = np.einsum("jin,in->jn", geo.JT, h)
    lhs = p @ sum(geo.Dv[j] @ W[j] for j in range(geo.d))
    rhs = -sum(np.sum(geo.J * h[i] * (geo.G[i] @ p)) for i in range(geo.d))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(p).sum())
    # the pin sees the boundary rows: a gradient with p_b = 0 in place of p_b = p_P breaks it
    assert geo.nb > 0
    bad = 0.0
    for f in range(geo.nb):
        P, j, s = geo.bP[f], geo.bj[f], geo.bs[f]
        # the (p_b - p_P) / 2 term with p_b = p_P vanishes; with p_b = 0 it is -p_P / 2 (sign N_f)
        bad += (2 * s - 1) * 0.5 * (-p[P]) * sum(geo.J[P] * h[i, P] * geo.T[j, i, P] for i in range(geo.d))
    assert abs(bad) > 1e-6 * (abs(lhs) + 1.0)
