"""Closed-form pin of a whole oracle step, both settings of the predictor's lagged
pressure (reading A2), in the Stokes limit (no GPU).

On a uniform periodic grid every operator of the step is diagonal on a Fourier mode
exp(i k . x): with spacing D, theta_j = k_j D, lambda = sum_j (2 - 2 cos theta_j) and
A = 1/dt + 4 nu / D^2 (alpha_jj = 1, J = D^2):

  C = 1/dt + nu lambda / D^2,  H = -(nu / D^2) sum_j 2 cos theta_j,
  grad: G_i = i sin(theta_i) / D,  div of lerp(J T h): sum_j i sin(theta_j) D h_j,
  pressure operator (faces lerp(alpha_jj / A)): -lambda / A.

The predictor solves C u* = u^n/dt + S (- G p^n with the switch); each corrector forms
h = (u^n/dt + S - H u) / A, solves -lambda/A p = div h and sets u = h - G p / A.  With a
velocity of 1e-10 the advective terms are 1e-10 of the result, so the step on one real
mode equals the real part of this scalar recurrence to that level.
"""
import math

import numpy as np
import pytest

import cases
from oracle.piso import Geometry, step


def _mode_step(k, dt, nu, D, u_hat, p_hat, S_hat, gradp, ncorr=2):
    th = np.array(k, dtype=float) * D
    lam = float(np.sum(2.0 - 2.0 * np.cos(th)))
    A = 1.0 / dt + 4.0 * nu / D ** 2
    Cs = 1.0 / dt + nu * lam / D ** 2
    Hs = -(nu / D ** 2) * float(np.sum(2.0 * np.cos(th)))
    G = 1j * np.sin(th) / D
    bu = u_hat / dt + S_hat
    b = bu - G * p_hat if gradp else bu
    u = b / Cs
    p = p_hat
    for _ in range(ncorr):
        h = (bu - Hs * u) / A
        rhs = np.sum(1j * np.sin(th) * D * h)
        p = rhs / (-lam / A)
        u = h - G * p / A
    return u, p


@pytest.mark.parametrize("gradp", [True, False])
@pytest.mark.parametrize("k", [(1, 0), (2, 3), (5, 2)])
def test_step_on_a_fourier_mode(k, gradp):
    n, nu, dt = 12, 0.05, 0.02
    case = cases.taylor_green(n, nu=nu, dt=dt)
    geo = Geometry(case.domain)
    D = 2 * math.pi / n
    x, y = case.domain.centres
    e = np.exp(1j * (k[0] * x + k[1] * y))
    eps = 1e-10
    u_hat = eps * np.array([1.0 + 0.5j, -0.3 + 0.2j])
    p_hat = 0.7 - 0.4j
    S_hat = np.array([0.3 + 0.1j, -0.2j])
    u_n = np.real(u_hat[:, None] * e[None])
    p_n = np.real(p_hat * e)
    S = np.real(S_hat[:, None] * e[None])
    rec = step(geo, u_n, p_n, nu, S, dt, case.u_b, grad_p_in_predictor=gradp)
    u1, p1 = _mode_step(k, dt, nu, D, u_hat, p_hat, S_hat, gradp)
    u_ref = np.real(u1[:, None] * e[None])
    p_ref = np.real(p1 * e)
    assert np.max(np.abs(rec.u2 - u_ref)) <= 1e-8 * np.max(np.abs(u_ref))
    assert np.max(np.abs(rec.p2 - p_ref)) <= 1e-8 * np.max(np.abs(p_ref))
    # the lagged pressure of the predictor changes the step (the pin sees the switch)
    u0, _ = _mode_step(k, dt, nu, D, u_hat, p_hat, S_hat, not gradp)
    assert np.max(np.abs(u1 - u0)) > 1e-6 * np.max(np.abs(u1))
