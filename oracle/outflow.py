"""FP64 oracle of the advective outflow boundary update and of its adjoint.

Test infrastructure: only tests, the smoke check and the benchmark's CPU baseline use
this module; the product path runs in the HIP library.

Between two PISO steps, the Dirichlet values on the faces marked as outflow are
advected out of the domain with a prescribed characteristic velocity u_m (App. A.4,
eq. advOut: du/dt + u_m du/dx = 0), and the updated outflow values are then scaled
so that the net volume flux through the boundary vanishes (the solver is
incompressible).  During the step the boundary is an ordinary Dirichlet boundary.

Readings (the printed update factor carries a sign that would make the scheme
anti-upwind for an outflow):
  * the face value is advanced implicitly, upwind from its boundary cell P, over the
    half-cell distance between the face and the cell centre:
        u_b* = (u_b + c u_P) / (1 + c),   c = 2 dt |T_j(P) . u_m|
    with j the face's axis and T_j(P) the contravariant row of the cell's metrics;
  * the flux of a boundary face is the one the step itself adds to the pressure
    right-hand side, U_b = N_b J_P T_j(P) . u_b (N_b = +1 on a high side, -1 on a low
    side); with Q_out the flux of the updated outflow faces and Q_rest that of all
    other Dirichlet faces, the outflow values are multiplied by s = -Q_rest / Q_out;
    when Q_out = 0 no scaling is applied (s = 1).

Parity: pinned by the closed-form geometric relaxation of a face value towards a
constant cell value, the zero net flux of the result, the reduction to plain implicit
upwinding when the fluxes already balance, and complex-step checks of the adjoint
(tests/test_oracle_outflow.py).
"""
from __future__ import annotations

import numpy as np

from .piso import Geometry


def face_coefficients(geo: Geometry, u_m, dt):
    """c_b = 2 dt |T_j(P) . u_m| of every Dirichlet face (the half cell from the boundary
    cell P) and the flux weights w_b = N_b (J T_j)_b of the face (shape [d, NB]), the
    weights of the Dirichlet flux the step adds to the pressure right-hand side."""
    u_m = np.asarray(u_m, dtype=np.float64)
    Tj = geo.T[geo.bj, :, geo.bP].T           # [d, NB]: T[j_b, i, P_b]
    c = 2.0 * dt * np.abs(np.einsum("in,i->n", Tj, u_m))
    w = geo.bN[None, :] * geo.bJT
    return c, w


def update(geo: Geometry, u_n, u_b, outflow, u_m, dt):
    """Updated Dirichlet values [d, NB] for the next step; u_n [d, N], u_b [d, NB],
    outflow a boolean mask [NB]."""
    outflow = np.asarray(outflow, dtype=bool)
    c, w = face_coefficients(geo, u_m, dt)
    uP = u_n[:, geo.bP]
    star = np.where(outflow[None, :], (u_b + c[None, :] * uP) / (1.0 + c[None, :]), u_b)
    q_out = np.sum(w[:, outflow] * star[:, outflow])
    q_rest = np.sum(w[:, ~outflow] * star[:, ~outflow])
    s = -q_rest / q_out if q_out != 0 else 1.0
    return np.where(outflow[None, :], s * star, star)


def update_vjp(geo: Geometry, u_n, u_b, outflow, u_m, dt, gbar):
    """Gradients (du_n [d, N], du_b [d, NB]) of <gbar, update(u_n, u_b)>."""
    outflow = np.asarray(outflow, dtype=bool)
    c, w = face_coefficients(geo, u_m, dt)
    uP = u_n[:, geo.bP]
    star = np.where(outflow[None, :], (u_b + c[None, :] * uP) / (1.0 + c[None, :]), u_b)
    q_out = np.sum(w[:, outflow] * star[:, outflow])
    q_rest = np.sum(w[:, ~outflow] * star[:, ~outflow])
    dtype = np.result_type(u_n, u_b, gbar)
    if q_out != 0:
        s = -q_rest / q_out
        sigma = np.sum(gbar[:, outflow] * star[:, outflow])     # d<gbar, out>/ds
        # s = -q_rest / q_out:  ds/dq_rest = -1/q_out,  ds/dq_out = -s/q_out
        star_bar = np.where(outflow[None, :], s * gbar - (sigma * s / q_out) * w,
                            gbar - (sigma / q_out) * w)
    else:
        star_bar = gbar.astype(dtype)
    du_b = np.where(outflow[None, :], star_bar / (1.0 + c[None, :]), star_bar)
    du_n = np.zeros(u_n.shape, dtype=dtype)
    contrib = np.where(outflow[None, :], star_bar * (c / (1.0 + c))[None, :], 0.0)
    for i in range(geo.d):
        np.add.at(du_n[i], geo.bP, contrib[i])
    return du_n, du_b
