"""Pins of the oracle adjoint (no GPU).

* complex-step directional derivatives (the forward oracle is analytic in its inputs
  with direct solves) against the hand-written vector-Jacobian product, on single and
  multi-block, orthogonal and sheared grids, 2D and 3D: |<Jv, w> - <v, J^T w>| tiny;
* central finite differences on a larger grid;
* the step is affine in the source S, so a finite change of S is predicted exactly
  by the S-gradient;
* a two-step rollout chains step gradients;
* the gradient-path flags of Sec. 2.4: each skipped adjoint solve equals the complex
  step of a forward whose corresponding solution is frozen (a stop-gradient).
"""
import numpy as np
import pytest

import cases
from oracle.adjoint import step_vjp
from oracle.piso import Geometry, step
from tests.test_oracle_pins import _two_block


def _state(case, seed):
    rng = np.random.default_rng(seed)
    d, N = case.u0.shape
    u = case.u0 + 0.2 * rng.standard_normal((d, N))
    p = rng.standard_normal(N)
    S = rng.standard_normal((d, N))
    ub = case.u_b + 0.1 * rng.standard_normal(case.u_b.shape)
    nu = case.nu * (1.0 + 0.2 * rng.random(N))
    return u, p, S, ub, nu


CASES = [
    lambda: cases.taylor_green(6, dt=0.2),
    lambda: cases.lid_cavity(6, n_steps=1),
    lambda: cases.channel(4, 5, 3),
    _two_block,
    lambda: cases.sheared_channel(5, 6, shear=0.8),
    lambda: cases.cylinder_oh(8, 4, 3),
]


@pytest.mark.parametrize("idx", range(len(CASES)))
@pytest.mark.parametrize("gradp", [True, False])
def test_complex_step_vjp(idx, gradp):
    case = CASES[idx]()
    geo = Geometry(case.domain)
    u, p, S, ub, nu = _state(case, 100 + idx)
    rng = np.random.default_rng(200 + idx)
    rec = step(geo, u, p, nu, S, case.dt, ub, grad_p_in_predictor=gradp)
    wu = rng.standard_normal(u.shape)
    wp = rng.standard_normal(p.shape)
    g = step_vjp(geo, rec, wu, wp)
    v = [rng.standard_normal(x.shape) for x in (u, p, S, ub)] + [case.nu * rng.standard_normal(nu.shape)]
    h = 1e-30
    rc = step(geo, u + 1j * h * v[0], p + 1j * h * v[1], nu + 1j * h * v[4], S + 1j * h * v[2],
              case.dt, ub + 1j * h * v[3], grad_p_in_predictor=gradp)
    jv = (np.sum(wu * rc.u2.imag) + np.sum(wp * rc.p2.imag)) / h
    vjp = (np.sum(g["u_n"] * v[0]) + np.sum(g["p_n"] * v[1]) + np.sum(g["S"] * v[2])
           + np.sum(g["u_b"] * v[3]) + np.sum(g["nu"] * v[4]))
    assert abs(jv - vjp) <= 1e-12 * abs(jv)


def test_central_fd_channel():
    case = cases.channel(8, 8, 8)
    geo = Geometry(case.domain)
    u, p, S, ub, nu = _state(case, 7)
    rng = np.random.default_rng(8)
    wu = rng.standard_normal(u.shape)
    rec = step(geo, u, p, case.nu, S, case.dt, ub)
    g = step_vjp(geo, rec, wu, np.zeros_like(p))
    for comp, cell in [(0, 5), (1, 77), (2, 300), (0, 511)]:
        eps = 1e-6 * max(1.0, abs(u[comp, cell]))
        up, um = u.copy(), u.copy()
        up[comp, cell] += eps
        um[comp, cell] -= eps
        fp = np.sum(wu * step(geo, up, p, case.nu, S, case.dt, ub).u2)
        fm = np.sum(wu * step(geo, um, p, case.nu, S, case.dt, ub).u2)
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g["u_n"][comp, cell]) <= 1e-6 * max(abs(fd), 1e-3)


def test_affine_in_source():
    """C, A and P do not depend on S: a finite change of S is predicted exactly."""
    case = cases.channel(6, 8, 6)
    geo = Geometry(case.domain)
    rng = np.random.default_rng(9)
    w = rng.standard_normal(case.u0.shape)
    rec = step(geo, case.u0, case.p0, case.nu, case.S, case.dt, case.u_b)
    g = step_vjp(geo, rec, w, np.zeros(geo.N))
    dS = 50.0 * rng.standard_normal(case.S.shape)
    rec2 = step(geo, case.u0, case.p0, case.nu, case.S + dS, case.dt, case.u_b)
    lhs = np.sum(w * (rec2.u2 - rec.u2))
    assert abs(lhs - np.sum(g["S"] * dS)) <= 1e-10 * abs(lhs)


def test_two_step_chain():
    case = cases.lid_cavity(6, n_steps=2)
    geo = Geometry(case.domain)
    u, p, S, ub, nu = _state(case, 11)
    rng = np.random.default_rng(12)
    w = rng.standard_normal(u.shape)
    r1 = step(geo, u, p, nu, S, case.dt, ub)
    r2 = step(geo, r1.u2, r1.p2, nu, S, case.dt, ub)
    g2 = step_vjp(geo, r2, w, np.zeros_like(p))
    g1 = step_vjp(geo, r1, g2["u_n"], g2["p_n"])
    dS = g1["S"] + g2["S"]
    v = rng.standard_normal(S.shape)
    h = 1e-30
    c1 = step(geo, u, p, nu, S + 1j * h * v, case.dt, ub)
    c2 = step(geo, c1.u2, c1.p2, nu, S + 1j * h * v, case.dt, ub)
    jv = np.sum(w * c2.u2.imag) / h
    assert abs(jv - np.sum(dS * v)) <= 1e-12 * abs(jv)


def test_gradient_path_flags_are_partial_sums():
    """Dropping both adjoint solves leaves only the bypass paths; results differ from the
    full gradient but stay finite, and dropping none reproduces the full gradient."""
    case = cases.taylor_green(6, dt=0.2)
    geo = Geometry(case.domain)
    u, p, S, ub, nu = _state(case, 13)
    rec = step(geo, u, p, nu, S, case.dt, ub)
    w = np.random.default_rng(14).standard_normal(u.shape)
    full = step_vjp(geo, rec, w, np.zeros_like(p))
    none = step_vjp(geo, rec, w, np.zeros_like(p), skip_velocity_solve=True, skip_pressure_solve=True)
    assert np.all(np.isfinite(none["u_n"]))
    assert np.linalg.norm(none["u_n"] - full["u_n"]) > 1e-6 * np.linalg.norm(full["u_n"])
    # with both solves skipped only the bypass through h of both correctors is left:
    # dS = g2 + g1 with g2 = w / A and g1 = -(H^T g2) / A
    g2 = w / rec.A
    g1 = -np.stack([rec.H.T @ g2[i] for i in range(2)]) / rec.A
    assert np.max(np.abs(none["S"] - (g2 + g1))) < 1e-14 * np.max(np.abs(g2))


def _frozen_solve_step(monkeypatch, velocity, pressure):
    """The forward oracle with the chosen linear solves taken as constants under the
    complex step: the solve is applied to the real parts of its operator and right-hand
    side only, so its solution carries no imaginary part (a stop-gradient)."""
    import oracle.piso as op
    sv, spr = op.solve_velocity, op.solve_pressure
    if velocity:
        monkeypatch.setattr(op, "solve_velocity",
                            lambda H, A, b, mode="direct", rtol=1e-13, x0=None, lu=None:
                            sv(H.real, A.real, b.real, mode, rtol))
    if pressure:
        monkeypatch.setattr(op, "solve_pressure",
                            lambda Pm, rhs, mode="direct", rtol=1e-13, x0=None:
                            spr(Pm.real, rhs.real, mode, rtol))
    return op.step


@pytest.mark.parametrize("idx", range(len(CASES)))
@pytest.mark.parametrize("flags", [1, 2, 3])
def test_gradient_path_flags_complex_step(monkeypatch, idx, flags):
    """Sec. 2.4 (eq. jnone): skipping the backward velocity solve (flag 1) is the gradient
    of the step with u* held constant, skipping the backward pressure solves (flag 2) the
    gradient with p* and p** held constant.  Pinned by the complex step of a forward in
    which exactly those solutions are frozen."""
    case = CASES[idx]()
    geo = Geometry(case.domain)
    u, p, S, ub, nu = _state(case, 300 + idx)
    rng = np.random.default_rng(400 + idx)
    rec = step(geo, u, p, nu, S, case.dt, ub)
    wu = rng.standard_normal(u.shape)
    wp = rng.standard_normal(p.shape)
    g = step_vjp(geo, rec, wu, wp, skip_velocity_solve=bool(flags & 1), skip_pressure_solve=bool(flags & 2))
    v = [rng.standard_normal(x.shape) for x in (u, p, S, ub)] + [case.nu * rng.standard_normal(nu.shape)]
    frozen = _frozen_solve_step(monkeypatch, bool(flags & 1), bool(flags & 2))
    h = 1e-30
    rc = frozen(geo, u + 1j * h * v[0], p + 1j * h * v[1], nu + 1j * h * v[4], S + 1j * h * v[2],
                case.dt, ub + 1j * h * v[3])
    jv = (np.sum(wu * rc.u2.imag) + np.sum(wp * rc.p2.imag)) / h
    vjp = (np.sum(g["u_n"] * v[0]) + np.sum(g["p_n"] * v[1]) + np.sum(g["S"] * v[2])
           + np.sum(g["u_b"] * v[3]) + np.sum(g["nu"] * v[4]))
    assert abs(jv - vjp) <= 1e-12 * abs(jv)
    # the frozen paths carry part of the full gradient, so the pin is not vacuous
    full = step_vjp(geo, rec, wu, wp)
    vjp_full = (np.sum(full["u_n"] * v[0]) + np.sum(full["p_n"] * v[1]) + np.sum(full["S"] * v[2])
                + np.sum(full["u_b"] * v[3]) + np.sum(full["nu"] * v[4]))
    assert abs(vjp_full - vjp) > 1e-6 * abs(vjp_full)
    # and each input's gradient on its own (a mistake confined to one input's path)
    for k, key in enumerate(("u_n", "p_n", "S", "u_b", "nu")):
        args = [u, p, S, ub, nu]
        args = [a + 1j * h * v[q] if q == k else a for q, a in enumerate(args)]
        r1 = frozen(geo, args[0], args[1], args[4], args[2], case.dt, args[3])
        jv_k = (np.sum(wu * r1.u2.imag) + np.sum(wp * r1.p2.imag)) / h
        vjp_k = np.sum(g[key] * v[k])
        assert abs(jv_k - vjp_k) <= 1e-12 * max(abs(jv), 1e-300), key
