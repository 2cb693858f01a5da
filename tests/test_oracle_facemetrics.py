"""Pins of the oracle's metrics on Dirichlet faces (no GPU).

A prescribed boundary carries its values and its metrics on the boundary face itself
(App. A.4), so the Dirichlet terms of the predictor (eq. velRHSdiscrete, the 2 alpha nu
diagonal of eq. difMatDiscrete, the deferred cross terms of eq. velRHSnonOrtho) and the
Dirichlet flux of the pressure right-hand side use the face's J and T when they are
given (Domain.Tb, Domain.Jb), and the boundary cell's otherwise.

* face metrics equal to the boundary cell's reproduce the default bit for bit;
* steady plane Couette flow by pure diffusion has a closed-form discrete solution (a
  constant flux through a chain of face conductances) that a wall-face alpha different
  from the cell's must reproduce, on a stretched grid;
* the pressure right-hand side sums to the net Dirichlet flux sum_f N_f (J T_j)_f . u_b
  taken from the face metrics (the interior and cross fluxes telescope);
* the adjoint with face metrics against complex steps of the forward;
* the outflow update balances the Dirichlet flux of the face metrics to zero.
"""
import dataclasses

import numpy as np
import pytest

import cases
from oracle import outflow as oout
from oracle.adjoint import step_vjp
from oracle.piso import (Geometry, assemble_C, h_and_rhs, predictor_rhs, solve_velocity, step)
from tests.test_oracle_adjoint import _state


def _with_face_metrics(case, seed, cross=0.15, Tb=None, Jb=None):
    """The case with face metrics: the boundary cells' values scaled at random, plus
    cross terms (cross > 0), unless Tb / Jb are given."""
    geo = Geometry(case.domain)
    d, nb = case.domain.dim, geo.nb
    rng = np.random.default_rng(seed)
    if Tb is None:
        Tb = geo.T[:, :, geo.bP] * (0.7 + 0.6 * rng.random((d, d, nb)))
        scale = np.abs(geo.T[:, :, geo.bP]).max(axis=(0, 1))
        Tb = Tb + cross * scale[None, None] * rng.standard_normal((d, d, nb)) * (1.0 - np.eye(d))[:, :, None]
    if Jb is None:
        Jb = geo.J[geo.bP] * (0.7 + 0.6 * rng.random(nb))
    dom = dataclasses.replace(case.domain, Tb=Tb, Jb=Jb)
    return dataclasses.replace(case, domain=dom)


NONORTH = [lambda: cases.sheared_channel(5, 6, shear=0.8), lambda: cases.cylinder_oh(8, 4, 3),
           lambda: cases.channel(4, 5, 3)]


@pytest.mark.parametrize("idx", range(len(NONORTH)))
def test_cell_values_on_faces_change_nothing(idx):
    case = NONORTH[idx]()
    geo0 = Geometry(case.domain)
    same = _with_face_metrics(case, 0, Tb=geo0.T[:, :, geo0.bP].copy(), Jb=geo0.J[geo0.bP].copy())
    u, p, S, ub, nu = _state(case, 40 + idx)
    r0 = step(geo0, u, p, nu, S, case.dt, ub)
    r1 = step(Geometry(same.domain), u, p, nu, S, case.dt, ub)
    assert np.array_equal(r0.u2, r1.u2) and np.array_equal(r0.p2, r1.p2)


def test_couette_closed_form_with_wall_face_metrics():
    """Walls at y = 0, 1 moving at -U and +U, periodic x, no forcing: the steady predictor
    (dt -> infinity, u^n = 0) is the discrete Couette profile.  Every y-face carries the
    same flux q: nu lerp(alpha_yy)_f (u_k+1 - u_k) inside, 2 nu alpha_b (u_1 - u_bottom) and
    2 nu alpha_b (u_top - u_ny) at the walls, so u_top - u_bottom fixes q."""
    nx, ny, U, nu = 3, 9, 1.5, 0.7
    xv = np.linspace(0.0, 1.0, nx + 1)
    yv = cases.tanh_vertices(ny, 1.4, 0.0, 1.0)
    T, J, c = cases.tensor_metrics([xv, yv])
    sides = cases.periodic_sides(0, 2, (0,)) + [cases.Side(0, 2, cases.DIRICHLET), cases.Side(0, 3, cases.DIRICHLET)]
    dom = cases.Domain(2, [(nx, ny, 1)], sides, T, J, c)
    ub = cases.boundary_values(dom, lambda si: np.array([-U if si == 2 else U, 0.0]) if si >= 2 else np.zeros(2))
    geo0 = Geometry(dom)
    nb = geo0.nb
    # wall-face metrics unlike the wall cells' (one factor per wall, so that every column
    # carries the same profile and no flux crosses the x-faces)
    top = geo0.bs == 1
    Tb = np.zeros((2, 2, nb))
    Tb[0, 0] = geo0.T[0, 0, geo0.bP]
    Tb[1, 1] = geo0.T[1, 1, geo0.bP] * np.where(top, 1.7, 2.3)
    Jb = geo0.J[geo0.bP] * np.where(top, 0.6, 1.3)
    dom = dataclasses.replace(dom, Tb=Tb, Jb=Jb)
    geo = Geometry(dom)
    dt = 1e15
    u_n = np.zeros((2, geo.N))
    H, A = assemble_C(geo, u_n, nu, dt)
    b = predictor_rhs(geo, u_n, nu, np.zeros((2, geo.N)), dt, ub)
    us, _ = solve_velocity(H, A, b)
    alpha_yy = J * T[1, 1] ** 2                          # alpha_jj = J T_j . T_j, cell centres
    alpha_b = Jb * (Tb[1, 0] ** 2 + Tb[1, 1] ** 2)       # the same on the faces
    for i in range(nx):
        col = i + nx * np.arange(ny)                     # cells of column i, bottom to top
        fb = [f for f in range(nb) if geo.bP[f] == col[0] and geo.bj[f] == 1][0]
        ft = [f for f in range(nb) if geo.bP[f] == col[-1] and geo.bj[f] == 1][0]
        res = np.r_[1.0 / (2 * nu * alpha_b[fb]),
                    1.0 / (nu * 0.5 * (alpha_yy[col[:-1]] + alpha_yy[col[1:]])),
                    1.0 / (2 * nu * alpha_b[ft])]           # resistances in series
        q = (U - (-U)) / res.sum()
        u_exact = -U + q * np.cumsum(res)[:-1]
        assert np.max(np.abs(us[0, col] - u_exact)) <= 1e-12 * U
        assert np.max(np.abs(us[1, col])) <= 1e-12 * U


@pytest.mark.parametrize("idx", range(len(NONORTH)))
def test_rhs_sums_to_the_face_flux(idx):
    case = _with_face_metrics(NONORTH[idx](), 10 + idx)
    geo = Geometry(case.domain)
    u, p, S, ub, nu = _state(case, 50 + idx)
    H, A = assemble_C(geo, u, nu, case.dt)
    b_u = predictor_rhs(geo, u, nu, S, case.dt, ub)
    _, rhs = h_and_rhs(geo, H, A, b_u, u, ub, p)
    Tb, Jb = case.domain.Tb, case.domain.Jb
    flux = sum((2.0 * geo.bs[f] - 1.0) * Jb[f] * Tb[geo.bj[f], :, f] @ ub[:, f] for f in range(geo.nb))
    assert abs(rhs.sum() - flux) <= 1e-12 * (np.abs(rhs).sum() + abs(flux))
    assert abs(flux) > 1e-3   # the test sees the face flux


@pytest.mark.parametrize("idx", range(len(NONORTH)))
def test_complex_step_vjp_with_face_metrics(idx):
    case = _with_face_metrics(NONORTH[idx](), 20 + idx)
    geo = Geometry(case.domain)
    assert geo.non_orthogonal
    u, p, S, ub, nu = _state(case, 60 + idx)
    rng = np.random.default_rng(70 + idx)
    rec = step(geo, u, p, nu, S, case.dt, ub)
    wu, wp = rng.standard_normal(u.shape), rng.standard_normal(p.shape)
    g = step_vjp(geo, rec, wu, wp)
    v = [rng.standard_normal(x.shape) for x in (u, p, S, ub)] + [case.nu * rng.standard_normal(nu.shape)]
    h = 1e-30
    rc = step(geo, u + 1j * h * v[0], p + 1j * h * v[1], nu + 1j * h * v[4], S + 1j * h * v[2], case.dt,
              ub + 1j * h * v[3])
    jv = (np.sum(wu * rc.u2.imag) + np.sum(wp * rc.p2.imag)) / h
    vjp = (np.sum(g["u_n"] * v[0]) + np.sum(g["p_n"] * v[1]) + np.sum(g["S"] * v[2])
           + np.sum(g["u_b"] * v[3]) + np.sum(g["nu"] * v[4]))
    assert abs(jv - vjp) <= 1e-12 * abs(jv)


def test_outflow_balances_the_face_flux():
    case = _with_face_metrics(cases.open_channel(8, 6), 30, cross=0.0)
    geo = Geometry(case.domain)
    rng = np.random.default_rng(31)
    u_n = case.u0 + 0.1 * rng.standard_normal(case.u0.shape)
    ub = case.u_b + 0.05 * rng.standard_normal(case.u_b.shape)
    new = oout.update(geo, u_n, ub, case.extra["outflow"], case.extra["u_m"], case.dt)
    Tb, Jb = case.domain.Tb, case.domain.Jb
    net = sum((2.0 * geo.bs[f] - 1.0) * Jb[f] * Tb[geo.bj[f], :, f] @ new[:, f] for f in range(geo.nb))
    inflow = sum(abs(Jb[f] * Tb[geo.bj[f], :, f] @ new[:, f]) for f in range(geo.nb))
    assert abs(net) <= 1e-13 * inflow
