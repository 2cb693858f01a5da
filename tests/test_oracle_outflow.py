"""Pins of the advective outflow oracle (App. A.4, eq. advOut; readings in
oracle/outflow.py)."""
import numpy as np
import pytest

import cases
from oracle import outflow
from oracle.piso import Geometry


def _open(nx=6, ny=5):
    case = cases.open_channel(nx, ny, length=3.0)
    return case, Geometry(case.domain)


def test_face_coefficients_closed_form():
    """On a uniform Cartesian x-spacing h the outflow faces get c = 2 dt |u_m,x| / h and
    the flux weight +J (high side), the inflow faces -J."""
    case, geo = _open()
    h = 3.0 / 6
    c, w = outflow.face_coefficients(geo, [0.7, -0.3], 0.05)
    mask = case.extra["outflow"]
    assert np.allclose(c[mask], 2 * 0.05 * 0.7 / h, rtol=1e-14)
    Jb = case.domain.J[geo.bP]
    inflow = cases.segment_mask(case.domain, lambda si: si == 0)
    assert np.allclose(w[0, mask], Jb[mask] / h) and np.allclose(w[1, mask], 0.0)
    assert np.allclose(w[0, inflow], -Jb[inflow] / h)


def test_geometric_relaxation_of_tangential_component():
    """With balanced normal fluxes (s = 1) the tangential outflow value relaxes towards a
    constant cell value as U + (V - U) (1 + c)^-n (implicit upwinding, solved by hand)."""
    case, geo = _open()
    mask = case.extra["outflow"]
    u_n = case.u0.copy()
    u_n[1] = 0.25                                      # uniform cross-stream velocity
    ub = case.u_b.copy()
    ub[1, mask] = -1.0
    u_m, dt = case.extra["u_m"], case.dt
    c = 2 * dt * u_m[0] / (3.0 / 6)
    for n in range(1, 6):
        ub = outflow.update(geo, u_n, ub, mask, u_m, dt)
        assert np.allclose(ub[1, mask], 0.25 + (-1.0 - 0.25) * (1 + c) ** (-n), rtol=0, atol=1e-14)
        # the streamwise value equals the cell value already: unchanged, s = 1
        assert np.allclose(ub[0, mask], case.u_b[0, mask], rtol=1e-14)


def test_zero_net_flux_and_identity_without_outflow():
    case, geo = _open(7, 6)
    rng = np.random.default_rng(1)
    u_n = rng.standard_normal(case.u0.shape)
    ub = rng.standard_normal(case.u_b.shape)
    mask = case.extra["outflow"]
    out = outflow.update(geo, u_n, ub, mask, [1.3, 0.2], 0.04)
    _, w = outflow.face_coefficients(geo, [1.3, 0.2], 0.04)
    assert abs(np.sum(w * out)) < 1e-13 * np.sum(np.abs(w * out))
    assert np.array_equal(out[:, ~mask], ub[:, ~mask])
    none = np.zeros_like(mask)
    assert np.array_equal(outflow.update(geo, u_n, ub, none, [1.3, 0.2], 0.04), ub)


def test_brute_force_loop():
    """Per-face loops with the metrics read straight from the domain."""
    case, geo = _open(5, 4)
    dom = case.domain
    rng = np.random.default_rng(2)
    u_n = rng.standard_normal(case.u0.shape)
    ub = rng.standard_normal(case.u_b.shape)
    mask = case.extra["outflow"]
    u_m, dt = np.array([0.9, 0.4]), 0.07
    star = ub.copy()
    q_out = q_rest = 0.0
    for b in range(ub.shape[1]):
        P, j, s = int(geo.bP[b]), int(geo.bj[b]), int(geo.bs[b])
        sign = 1.0 if s == 1 else -1.0
        tj = [dom.T[j, i, P] for i in range(2)]
        if mask[b]:
            cc = 2 * dt * abs(tj[0] * u_m[0] + tj[1] * u_m[1])
            for i in range(2):
                star[i, b] = (ub[i, b] + cc * u_n[i, P]) / (1 + cc)
        flux = sign * dom.J[P] * (tj[0] * star[0, b] + tj[1] * star[1, b])
        if mask[b]:
            q_out += flux
        else:
            q_rest += flux
    ref = star.copy()
    ref[:, mask] *= -q_rest / q_out
    assert np.allclose(outflow.update(geo, u_n, ub, mask, u_m, dt), ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("which", ["open", "cylinder"])
def test_vjp_complex_step(which):
    if which == "open":
        case, geo = _open(6, 5)
        mask = case.extra["outflow"]
    else:
        case = cases.cylinder_oh(16, 6, 5)
        geo = Geometry(case.domain)
        # outflow on the +x side of the box (transition block 1, outer side)
        mask = cases.segment_mask(case.domain, lambda si: case.domain.sides[si].block == 1)
    rng = np.random.default_rng(3)
    u_n = rng.standard_normal(case.u0.shape)
    ub = rng.standard_normal(case.u_b.shape) + 1.0
    gbar = rng.standard_normal(ub.shape)
    u_m, dt = [1.1, -0.2], 0.03
    du_n, du_b = outflow.update_vjp(geo, u_n, ub, mask, u_m, dt, gbar)
    for seed in range(3):
        r = np.random.default_rng(10 + seed)
        vn, vb = r.standard_normal(u_n.shape), r.standard_normal(ub.shape)
        hh = 1e-30
        out = outflow.update(geo, u_n + 1j * hh * vn, ub + 1j * hh * vb, mask, u_m, dt)
        cs = np.sum(gbar * out.imag) / hh
        an = np.sum(du_n * vn) + np.sum(du_b * vb)
        assert abs(cs - an) <= 1e-12 * max(1.0, abs(an))
