"""Pins of the divergence-free gradient modification oracle (eq. SgradPsgrad)."""
import numpy as np
import pytest

import cases
from oracle.divfree import divfree_gradient
from oracle.piso import Geometry, face_flux_divergence
from tests.test_oracle_pins import _two_block


def _geos():
    return {"tgv": cases.taylor_green(8).domain, "channel": cases.channel(6, 8, 5).domain,
            "two_block": _two_block().domain, "cylinder": cases.cylinder_oh(16, 6, 5).domain,
            "sheared": cases.sheared_channel(6, 7, shear=0.5).domain}


@pytest.mark.parametrize("name", list(_geos()))
def test_projected_source_is_divergence_free(name):
    dom = _geos()[name]
    geo = Geometry(dom)
    rng = np.random.default_rng(7)
    S = rng.standard_normal((geo.d, geo.N))
    g, p = divfree_gradient(geo, S, np.zeros_like(S), 1.0)
    assert np.allclose(g, geo.grad(p), rtol=0, atol=0)
    div = face_flux_divergence(geo, S, np.ones(geo.N), p, np.zeros(geo.N), np.zeros((geo.d, geo.nb)))
    ref = face_flux_divergence(geo, S, np.ones(geo.N), np.zeros(geo.N), np.zeros(geo.N),
                               np.zeros((geo.d, geo.nb)))
    assert np.max(np.abs(div)) <= 1e-11 * np.max(np.abs(ref))
    assert abs(p.mean()) < 1e-13


def test_identity_and_linearity():
    geo = Geometry(cases.channel(6, 8, 5).domain)
    rng = np.random.default_rng(8)
    S1, S2, gS = (rng.standard_normal((geo.d, geo.N)) for _ in range(3))
    g0, _ = divfree_gradient(geo, S1, gS, 0.0)
    assert np.array_equal(g0, gS)
    a, _ = divfree_gradient(geo, S1, np.zeros_like(gS), 1.0)
    b, _ = divfree_gradient(geo, S2, np.zeros_like(gS), 1.0)
    c, _ = divfree_gradient(geo, 2.0 * S1 - 3.0 * S2, np.zeros_like(gS), 1.0)
    assert np.allclose(c, 2.0 * a - 3.0 * b, rtol=1e-10, atol=1e-12)
    d, _ = divfree_gradient(geo, S1, gS, 0.5)
    assert np.allclose(d, gS + 0.5 * a, rtol=1e-12, atol=1e-12)
