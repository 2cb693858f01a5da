"""FP64 oracle of the adjoint (vector-Jacobian product) of one PISO step.

Discretise-then-optimise through the step (Sec. 2.3 and App. A.5 of the paper), with
each linear solve differentiated as an adjoint solve: for A x = b the incoming
gradient dx gives db from A^T db = dx and dA = -db (x) x on the sparsity pattern of A.
Every other operation is the exact transpose of its forward linearisation; terms that
App. A.5 omits "for simplicity" (the non-orthogonal lags, the A-dependence of P through
its face coefficients) are kept, so that the result is the exact gradient of the
forward oracle.  Gradients are not taken with respect to the metrics or dt.

Parity: pinned by complex-step directional derivatives and dot-product tests on small
single- and multi-block, orthogonal and sheared grids (tests/test_oracle_adjoint.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .piso import Geometry, StepRecord, solve_pressure


def _cross_kappa_bar(geo: Geometry, phi, ybar):
    """d/d kappa of <ybar, K(kappa) phi> for the deferred cross operator."""
    out = np.zeros(geo.N, dtype=np.result_type(phi, ybar))
    g = np.stack([geo.Gt[k] @ phi for k in range(geo.d)])
    for j in range(geo.d):
        P, F = geo.faces[j]
        dy = ybar[P] - ybar[F]
        for k in range(geo.d):
            if k == j:
                continue
            t = 0.5 * (g[k, P] + g[k, F])
            np.add.at(out, P, 0.5 * geo.alpha[j, k, P] * t * dy)
            np.add.at(out, F, 0.5 * geo.alpha[j, k, F] * t * dy)
    return out


class _Grads:
    def __init__(self, geo, dtype):
        d, N = geo.d, geo.N
        self.A = np.zeros(N, dtype=dtype)
        self.Hpf = [np.zeros(len(geo.faces[j][0]), dtype=dtype) for j in range(d)]  # dC[P,F]
        self.Hfp = [np.zeros(len(geo.faces[j][0]), dtype=dtype) for j in range(d)]  # dC[F,P]
        self.b_u = np.zeros((d, N), dtype=dtype)
        self.u_n = np.zeros((d, N), dtype=dtype)
        self.p_n = np.zeros(N, dtype=dtype)
        self.S = np.zeros((d, N), dtype=dtype)
        self.nu = np.zeros(N, dtype=dtype)
        self.u_b = np.zeros((d, geo.nb), dtype=dtype)


def _outer_on_pattern(geo, G, left, right):
    """Accumulate -sum_i left_i[P] right_i[F] into the off-diagonal pattern of C."""
    for j in range(geo.d):
        P, F = geo.faces[j]
        G.Hpf[j] -= np.einsum("in,in->n", left[:, P], right[:, F])
        G.Hfp[j] -= np.einsum("in,in->n", left[:, F], right[:, P])


def correct_vjp(geo, G, A, p, ubar):
    """u = h - A^-1 grad p: returns (hbar, pbar) and accumulates dA."""
    gp = geo.grad(p)
    G.A += np.sum(gp * ubar, axis=0) / A ** 2
    g = ubar / A
    pbar = -sum(geo.G[i].T @ g[i] for i in range(geo.d))
    return ubar.copy(), pbar


def pressure_solve_vjp(geo, G, rec, A, p, pbar, mode, rtol):
    """p = zero-mean solution of P p = rhs - mean(rhs): lambda = P^+ pbar, rhs_bar =
    lambda; dP = -lambda (x) p mapped to the face coefficients and then to dA."""
    lam = solve_pressure(rec.Pm, pbar, mode, rtol)
    for j in range(geo.d):
        P, F = geo.faces[j]
        pfbar = (lam[P] - lam[F]) * (p[P] - p[F])
        np.add.at(G.A, P, pfbar * (-0.5 * geo.alpha[j, j, P] / A[P] ** 2))
        np.add.at(G.A, F, pfbar * (-0.5 * geo.alpha[j, j, F] / A[F] ** 2))
    return lam


def h_rhs_vjp(geo, G, rec, A, h, u_in, p_lag, hbar, rhsbar):
    """Adjoint of h = A^-1 (b_u - H u_in) and rhs = div(J T h) + Dirichlet flux
    - K(1/A) p_lag.  Returns (u_in_bar, p_lag_bar); accumulates dA, dH, db_u, du_b."""
    d = geo.d
    Wbar = np.stack([geo.Dv[j].T @ rhsbar for j in range(d)])
    hbar = hbar + np.einsum("jin,jn->in", geo.JT, Wbar)
    if geo.nb:
        for i in range(d):
            G.u_b[i] += geo.Bflux[i].T @ rhsbar
    p_lag_bar = np.zeros(geo.N, dtype=G.A.dtype)
    if geo.non_orthogonal:
        kap = 1.0 / A
        K = geo.cross_operator(kap)
        p_lag_bar = p_lag_bar - K.T @ rhsbar
        kbar = _cross_kappa_bar(geo, p_lag, -rhsbar)
        G.A += kbar * (-1.0 / A ** 2)
    g = hbar / A
    G.b_u += g
    H = rec.H
    u_in_bar = -np.stack([H.T @ g[i] for i in range(d)])
    _outer_on_pattern(geo, G, g, u_in)
    G.A += -np.sum(hbar * h, axis=0) / A
    return u_in_bar, p_lag_bar


def step_vjp(geo: Geometry, rec: StepRecord, ubar, pbar, mode="direct", rtol=1e-13,
             skip_velocity_solve=False, skip_pressure_solve=False):
    """Gradients of <ubar, u^{n+1}> + <pbar, p^{n+1}> with respect to u^n, p^n, S, nu
    (per cell), and u_b.  Returns a dict of arrays.

    skip_* drop the adjoint linear solves (the approximate gradient paths of Sec. 2.4):
    the corresponding adjoint solution is taken as zero.
    """
    d = geo.d
    dtype = np.result_type(rec.u2, ubar, pbar)
    G = _Grads(geo, dtype)
    A = rec.A
    # corrector 2 then corrector 1
    hs = [rec.h1, rec.h2]
    ps = [rec.p1, rec.p2]
    u_ins = [rec.u_star, rec.u1]
    p_lags = [rec.p_n, rec.p1]
    uc_bar = np.asarray(ubar, dtype=dtype)
    pc_bar = np.asarray(pbar, dtype=dtype).copy()
    p_lag_extra = np.zeros(geo.N, dtype=dtype)
    for c in (1, 0):
        hbar, pb = correct_vjp(geo, G, A, ps[c], uc_bar)
        pc_total = pc_bar + pb
        if skip_pressure_solve:
            rhsbar = np.zeros(geo.N, dtype=dtype)
        else:
            rhsbar = pressure_solve_vjp(geo, G, rec, A, ps[c], pc_total, mode, rtol)
        u_in_bar, p_lag_bar = h_rhs_vjp(geo, G, rec, A, hs[c], u_ins[c], p_lags[c], hbar, rhsbar)
        uc_bar = u_in_bar
        if c == 1:
            pc_bar = p_lag_bar          # flows into p* (the lag of corrector 2)
        else:
            p_lag_extra = p_lag_bar     # flows into p^n (the lag of corrector 1)
    G.p_n += p_lag_extra
    ustar_bar = uc_bar
    # velocity solve: mu = C^-T ustar_bar, db = mu, dC = -mu (x) u*
    if skip_velocity_solve:
        mu = np.zeros_like(ustar_bar)
    else:
        C = (rec.H + sp.diags(A)).tocsc()
        if mode == "direct":
            lu = rec.lu if rec.lu is not None and np.result_type(rec.lu.U.dtype, dtype) == rec.lu.U.dtype \
                else spla.splu(C.astype(dtype))
            mu = np.stack([lu.solve(ustar_bar[i], trans="T") for i in range(d)])
        else:
            mu = []
            for i in range(d):
                x, info = spla.bicgstab(C.T.tocsr(), ustar_bar[i], rtol=rtol, atol=0.0, maxiter=20000)
                if info != 0:
                    raise RuntimeError("oracle adjoint BiCGStab did not converge")
                mu.append(x)
            mu = np.stack(mu)
        _outer_on_pattern(geo, G, mu, rec.u_star)
        G.A += -np.sum(mu * rec.u_star, axis=0)
    # b = b_u - grad p^n
    G.b_u += mu
    if rec.grad_p_in_predictor:
        G.p_n += -sum(geo.G[i].T @ mu[i] for i in range(d))
    # b_u = u^n/dt + S + boundary terms + deferred cross diffusion
    nu, u_b, u_n, dt = rec.nu, rec.u_b, rec.u_n, rec.dt
    G.u_n += G.b_u / dt
    G.S += G.b_u
    if geo.nb:
        P, j = geo.bP, geo.bj
        JTb = geo.bJT                                 # [d, NB]
        Ub = np.einsum("in,in->n", JTb, u_b)
        coef = 2.0 * geo.balpha_jj * nu[P] - geo.bN * Ub
        bub = G.b_u[:, P]                              # [d, NB]
        G.u_b += bub * coef / geo.J[P]
        G.u_b += (-geo.bN / geo.J[P]) * JTb * np.sum(bub * u_b, axis=0)
        np.add.at(G.nu, P, np.sum(bub * u_b, axis=0) * 2.0 * geo.balpha_jj / geo.J[P])
    if geo.non_orthogonal:
        K = geo.cross_operator(nu)
        for i in range(d):
            y = G.b_u[i] / geo.J
            G.u_n[i] += K.T @ y
            G.nu += _cross_kappa_bar(geo, u_n[i], y)
            if geo.nb:
                yb = y[geo.bP]
                for k in range(d):
                    w = geo.bN * geo.balpha[k] * np.where(geo.bj == k, 0.0, 1.0)
                    G.u_b[i] += geo.Bt[k].T @ (w * nu[geo.bP] * yb)
                    np.add.at(G.nu, geo.bP, w * (geo.Bt[k] @ u_b[i]) * yb)
    # C and A from the face fluxes and nu (eqs. advMatDiscrete, difMatDiscrete)
    Ubar = np.zeros((d, geo.N), dtype=dtype)
    for j in range(d):
        P, F = geo.faces[j]
        JP, JF = geo.J[P], geo.J[F]
        phibar = 0.5 * G.Hpf[j] / JP - 0.5 * G.Hfp[j] / JF + 0.5 * G.A[P] / JP - 0.5 * G.A[F] / JF
        kbar = -G.Hpf[j] / JP - G.Hfp[j] / JF + G.A[P] / JP + G.A[F] / JF
        np.add.at(G.nu, P, 0.5 * geo.alpha[j, j, P] * kbar)
        np.add.at(G.nu, F, 0.5 * geo.alpha[j, j, F] * kbar)
        np.add.at(Ubar[j], P, 0.5 * phibar)
        np.add.at(Ubar[j], F, 0.5 * phibar)
    if geo.nb:
        np.add.at(G.nu, geo.bP, 2.0 * geo.balpha_jj * G.A[geo.bP] / geo.J[geo.bP])
    G.u_n += np.einsum("jin,jn->in", geo.JT, Ubar)
    return {"u_n": G.u_n, "p_n": G.p_n, "S": G.S, "nu": G.nu, "u_b": G.u_b,
            "A": G.A, "mu": mu}
