"""FP64 oracle of one PISO step (App. A.2-A.4 of the paper), written as explicit
sparse matrices and per-face loops that follow the printed discretisation.

One step, given u^n, p^n, viscosity nu, sources S, Dirichlet values u_b and dt:

  predictor (eq. advectionMat):  C(u^n) u* = b,  b = b_u - grad p^n
  corrector c = 1, 2 (eqs. pressureRHS, pressure, correction):
      h   = A^-1 (b_u - H u)                 u = u* for c = 1, u** for c = 2
      P p = div h (+ boundary flux, + deferred non-orthogonal term)
      u   = h - A^-1 grad p
  u^{n+1} = u***, p^{n+1} = p**

Readings of the paper adopted here (each also listed in the design document):
  * rows of C are per unit volume: temporal term 1/dt, face terms divided by J_P, so
    that the right-hand side of eq. velRHSdiscrete and the correction eq. velCorrDiscrete
    are in consistent units;
  * -grad p^n enters the predictor right-hand side only (eq. implEuler1); h excludes it;
  * grad p uses central differences in computational space with the boundary-face value
    p_b = p_P at a non-connected side (zero-Neumann pressure, App. A.4);
  * "lerp" is the arithmetic mean of the two cell values;
  * boundary-face metrics are those of the adjacent cell;
  * the divergence of h also carries the prescribed Dirichlet face flux;
  * non-orthogonal (alpha_jk, j != k) fluxes are fully deferred to the right-hand side
    (App. A.3.5) with lagged fields (u^n for the predictor, p^n and p* for the two
    correctors); the tangential derivative at a face is the mean of the two cells'
    central computational differences, one-sided next to a non-connected side;
  * the pressure system is singular (velocity-Dirichlet sides imply zero-Neumann
    pressure); its right-hand side is made zero-mean and the zero-mean solution is
    returned.

Parity: pinned by the tests in tests/test_oracle_*.py (dense brute force, plane
Poiseuille closed form, Taylor-Green linear decay factor and continuum decay, exact
Fourier symbols on a sheared periodic grid, divergence after correction, invariants).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from cases import Domain
from .topology import build_topology


def _csr(rows, cols, vals, n, m=None):
    m = n if m is None else m
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, m)).tocsr()


class Geometry:
    """State-independent data of a domain: adjacency, metrics and sparse stencils."""

    def __init__(self, dom: Domain):
        self.dom = dom
        topo = build_topology(dom)
        self.topo = topo
        d, N = dom.dim, topo.n_cells
        self.d, self.N = d, N
        self.T = np.asarray(dom.T, dtype=np.float64)
        self.J = np.asarray(dom.J, dtype=np.float64)
        # alpha_jk = J T_j . T_k  (App. A.3.3, diffusion term)
        self.alpha = self.J[None, None] * np.einsum("jin,kin->jkn", self.T, self.T)
        self.JT = self.J[None, None] * self.T
        nbr = topo.nbr
        cells = np.arange(N)
        # interior / connected faces, each listed once as the high face of its low cell
        self.faces = []
        for j in range(d):
            F = nbr[:, j, 1]
            m = F >= 0
            self.faces.append((cells[m], F[m]))
        self.nb = topo.n_bfaces
        self.bP, self.bj, self.bs = topo.bface_cell, topo.bface_axis, topo.bface_side
        self.bN = 2.0 * self.bs - 1.0          # outward face sign of each boundary face
        # metrics of the Dirichlet faces (App. A.4: a prescribed boundary carries its values
        # and metrics on the face itself); without them those of the boundary cell.
        # bJT[i, f] = J T_{j_f, i} (the face's own axis j_f), balpha[k, f] = alpha_{j_f k}
        fb = np.arange(self.nb)
        if getattr(dom, "Tb", None) is None:
            self.bJT = self.JT[self.bj, :, self.bP].T
            self.balpha = self.alpha[self.bj, :, self.bP].T
        else:
            Tb = np.asarray(dom.Tb, dtype=np.float64)
            Jb = np.asarray(dom.Jb, dtype=np.float64)
            if Tb.shape != (d, d, self.nb) or Jb.shape != (self.nb,) or not np.all(Jb > 0):
                raise ValueError("face metrics: Tb [d, d, NB] and Jb [NB] > 0 expected")
            alpha_b = Jb[None, None] * np.einsum("jib,kib->jkb", Tb, Tb)
            self.bJT = (Jb[None, None] * Tb)[self.bj, :, fb].T
            self.balpha = alpha_b[self.bj, :, fb].T
        self.balpha_jj = self.balpha[self.bj, fb]
        off = np.abs(self.alpha[~np.eye(d, dtype=bool)]) if d > 1 else np.zeros(1)
        diag = np.abs(self.alpha[np.eye(d, dtype=bool)]).min(axis=0)
        self.non_orthogonal = bool(np.max(off / diag) > 1e-12)
        if self.nb and d > 1:   # cross terms of the face metrics count too
            cross = np.abs(np.where(np.arange(d)[:, None] == self.bj[None, :], 0.0, self.balpha)).max(axis=0)
            self.non_orthogonal |= bool(np.max(cross / np.abs(self.balpha_jj)) > 1e-12)

        # pressure gradient: (grad p)_i = sum_j T_ji (p_{+j} - p_{-j}) / 2, p_b = p_P
        self.dcomp = []
        for j in range(d):
            Fp, Fm = nbr[:, j, 1], nbr[:, j, 0]
            cp = np.where(Fp >= 0, Fp, cells)
            cm = np.where(Fm >= 0, Fm, cells)
            self.dcomp.append(_csr(np.r_[cells, cells], np.r_[cp, cm],
                                   np.r_[0.5 * np.ones(N), -0.5 * np.ones(N)], N))
        self.G = [sum(sp.diags(self.T[j, i]) @ self.dcomp[j] for j in range(d)).tocsr()
                  for i in range(d)]

        # tangential computational derivative of a cell field (non-orthogonal terms)
        self.Gt = []
        for k in range(d):
            Fp, Fm = nbr[:, k, 1], nbr[:, k, 0]
            hp, hm = Fp >= 0, Fm >= 0
            both = hp & hm
            rows, cols, vals = [], [], []
            rows += [cells[both], cells[both]]
            cols += [Fp[both], Fm[both]]
            vals += [0.5 * np.ones(both.sum()), -0.5 * np.ones(both.sum())]
            only_p = hp & ~hm
            rows += [cells[only_p], cells[only_p]]
            cols += [Fp[only_p], cells[only_p]]
            vals += [np.ones(only_p.sum()), -np.ones(only_p.sum())]
            only_m = hm & ~hp
            rows += [cells[only_m], cells[only_m]]
            cols += [cells[only_m], Fm[only_m]]
            vals += [np.ones(only_m.sum()), -np.ones(only_m.sum())]
            self.Gt.append(_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), N))

        # divergence of a face-interpolated cell vector field W (eq. pressureRHSdivDiscrete)
        self.Dv = []
        for j in range(d):
            P, F = self.faces[j]
            h = 0.5 * np.ones(len(P))
            self.Dv.append(_csr(np.r_[P, P, F, F], np.r_[P, F, P, F], np.r_[h, h, -h, -h], N))

        # prescribed Dirichlet face flux N_b U_b(u_b), U_b = (J T_j)_b . u_b
        self.Bflux = []
        for i in range(d):
            v = self.bN * self.bJT[i]
            self.Bflux.append(_csr(self.bP, np.arange(self.nb), v, N, self.nb))

        # tangential derivative of boundary values along a Dirichlet side
        self.Bt = []
        bidx = -1 - nbr
        for k in range(d):
            rows, cols, vals = [], [], []
            for b in range(self.nb):
                P, j, s = self.bP[b], self.bj[b], self.bs[b]
                if k == j:
                    continue
                nb_ = []
                for side in (1, 0):
                    Q = nbr[P, k, side]
                    nb_.append(bidx[Q, j, s] if Q >= 0 and nbr[Q, j, s] < 0 else -1)
                bp, bm = nb_
                if bp >= 0 and bm >= 0:
                    rows += [b, b]; cols += [bp, bm]; vals += [0.5, -0.5]
                elif bp >= 0:
                    rows += [b, b]; cols += [bp, b]; vals += [1.0, -1.0]
                elif bm >= 0:
                    rows += [b, b]; cols += [b, bm]; vals += [1.0, -1.0]
            self.Bt.append(_csr(np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64),
                                np.array(vals), self.nb))

    # ------------------------------------------------------------------ helpers
    def nu_field(self, nu):
        nu = np.asarray(nu)
        return np.broadcast_to(nu, (self.N,)) if nu.ndim == 0 or nu.size == 1 else nu

    def contravariant(self, u):
        """U^j = J T_j . u at cell centres (App. A.3.2)."""
        return np.einsum("jin,in->jn", self.JT, u)

    def grad(self, p):
        return np.stack([G @ p for G in self.G])

    def cross_operator(self, kappa):
        """Sparse K(kappa) with (K phi)_P = sum_f N_f sum_{k != j} lerp(alpha_jk kappa)_f
        * (d phi / d xi^k)_f over the interior faces of P: the deferred non-orthogonal
        part of div(kappa grad phi) (App. A.3.5), volume-integrated."""
        N, d = self.N, self.d
        K = sp.csr_matrix((N, N), dtype=np.result_type(kappa, np.float64))
        for j in range(d):
            P, F = self.faces[j]
            nf = len(P)
            if nf == 0:
                continue
            SP = _csr(np.arange(nf), P, np.ones(nf), nf, N)
            SF = _csr(np.arange(nf), F, np.ones(nf), nf, N)
            scatter = (SP - SF).T
            for k in range(d):
                if k == j:
                    continue
                w = 0.5 * (self.alpha[j, k, P] * kappa[P] + self.alpha[j, k, F] * kappa[F])
                K = K + scatter @ sp.diags(w) @ (0.5 * (SP + SF)) @ self.Gt[k]
        return K.tocsr()

    def boundary_cross(self, nu, ub_i):
        """Deferred non-orthogonal flux through Dirichlet faces, N_b sum_k alpha_jk nu
        d(u_b)/d xi^k, scattered to the owning cells (volume-integrated)."""
        out = np.zeros(self.N, dtype=np.result_type(nu, ub_i, np.float64))
        if self.nb == 0:
            return out
        for k in range(self.d):
            gk = self.Bt[k] @ ub_i
            v = self.bN * self.balpha[k] * nu[self.bP] * gk
            v = np.where(self.bj == k, 0.0, v)
            np.add.at(out, self.bP, v)
        return out


# ---------------------------------------------------------------------- forward ops

def assemble_C(geo: Geometry, u_n, nu, dt):
    """Advection-diffusion matrix C = C^t + C^adv + C^nu with per-volume rows.

    Face flux U_f = (U_P + U_F)/2 (App. A.3.3, advection term); eq. advMatDiscrete gives
    the advective entries 0.5 N_f U_f, eq. difMatDiscrete the diffusive ones -lerp(alpha_jj nu)
    with 2 alpha_jj nu on the diagonal for a Dirichlet face.  Returns (H, A): the
    off-diagonal part and the diagonal of C.
    """
    N = geo.N
    nu = geo.nu_field(nu)
    U = geo.contravariant(u_n)
    dtype = np.result_type(u_n, nu, np.float64)
    A = np.full(N, 1.0 / dt, dtype=dtype)
    rows, cols, vals = [], [], []
    for j in range(geo.d):
        P, F = geo.faces[j]
        phi = 0.5 * (U[j, P] + U[j, F])
        knu = 0.5 * (geo.alpha[j, j, P] * nu[P] + geo.alpha[j, j, F] * nu[F])
        rows += [P, F]
        cols += [F, P]
        vals += [(0.5 * phi - knu) / geo.J[P], (-0.5 * phi - knu) / geo.J[F]]
        np.add.at(A, P, (0.5 * phi + knu) / geo.J[P])
        np.add.at(A, F, (-0.5 * phi + knu) / geo.J[F])
    if geo.nb:
        np.add.at(A, geo.bP, 2.0 * geo.balpha_jj * nu[geo.bP] / geo.J[geo.bP])
    H = _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals).astype(dtype), N)
    return H, A


def predictor_rhs(geo: Geometry, u_n, nu, S, dt, u_b):
    """b_u = u^n/dt + (1/J_P) sum_b u_b (2 alpha_jj nu - N_b U_b) + S  (eq. velRHSdiscrete)
    plus the deferred non-orthogonal diffusion of u^n and of u_b (eq. velRHSnonOrtho)."""
    nu = geo.nu_field(nu)
    b_u = u_n / dt + S
    b_u = b_u.astype(np.result_type(b_u, nu, u_b, np.float64))
    if geo.nb:
        Ub = np.einsum("in,in->n", geo.bJT, u_b)
        coef = 2.0 * geo.balpha_jj * nu[geo.bP] - geo.bN * Ub
        for i in range(geo.d):
            np.add.at(b_u[i], geo.bP, u_b[i] * coef / geo.J[geo.bP])
    if geo.non_orthogonal:
        K = geo.cross_operator(nu)
        for i in range(geo.d):
            b_u[i] += (K @ u_n[i] + geo.boundary_cross(nu, u_b[i])) / geo.J
    return b_u


def pressure_matrix(geo: Geometry, A):
    """P with P_F = lerp(alpha_jj / A), P_P = -sum_F P_F  (eq. pMatDiscrete)."""
    N = geo.N
    rows, cols, vals = [], [], []
    diag = np.zeros(N, dtype=A.dtype)
    for j in range(geo.d):
        P, F = geo.faces[j]
        pf = 0.5 * (geo.alpha[j, j, P] / A[P] + geo.alpha[j, j, F] / A[F])
        rows += [P, F]
        cols += [F, P]
        vals += [pf, pf]
        np.add.at(diag, P, -pf)
        np.add.at(diag, F, -pf)
    off = _csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), N)
    return (off + sp.diags(diag)).tocsr()


def h_and_rhs(geo: Geometry, H, A, b_u, u, u_b, p_lag):
    """h = A^-1 (b_u - H u) (eq. pressureRHS) and its divergence (eq.
    pressureRHSdivDiscrete) plus the Dirichlet face flux and the deferred
    non-orthogonal pressure term of p_lag (eq. pressureRHSnonOrtho)."""
    h = np.stack([(b_u[i] - H @ u[i]) / A for i in range(geo.d)])
    W = np.einsum("jin,in->jn", geo.JT, h)
    rhs = sum(geo.Dv[j] @ W[j] for j in range(geo.d))
    if geo.nb:
        rhs = rhs + sum(geo.Bflux[i] @ u_b[i] for i in range(geo.d))
    if geo.non_orthogonal:
        rhs = rhs - geo.cross_operator(1.0 / A) @ p_lag
    return h, rhs


def solve_pressure(Pm, rhs, mode="direct", rtol=1e-13, x0=None):
    """Zero-mean solution of the singular system P p = rhs - mean(rhs)."""
    N = Pm.shape[0]
    r = rhs - rhs.mean()
    if mode == "direct":
        ones = np.ones((N, 1))
        Mb = sp.bmat([[Pm, sp.csr_matrix(ones)], [sp.csr_matrix(ones.T), None]]).tocsc()
        dtype = np.result_type(Pm.dtype, r.dtype)
        lu = spla.splu(Mb.astype(dtype))
        p = lu.solve(np.r_[r, 0.0].astype(dtype))[:N]
    else:
        Mneg = (-Pm).tocsr()
        dinv = 1.0 / Mneg.diagonal()
        prec = spla.LinearOperator((N, N), matvec=lambda x: dinv * x, dtype=np.float64)
        p, info = spla.cg(Mneg, -r, x0=x0, rtol=rtol, atol=0.0, maxiter=20000, M=prec)
        if info != 0:
            raise RuntimeError("oracle CG did not converge (info=%d)" % info)
    return p - p.mean()


def solve_velocity(H, A, b, mode="direct", rtol=1e-13, x0=None, lu=None):
    C = (H + sp.diags(A)).tocsc()
    if mode == "direct":
        C = C.astype(np.result_type(C.dtype, b.dtype))
        lu = spla.splu(C) if lu is None else lu
        return np.stack([lu.solve(bi) for bi in b]), lu
    out = []
    for i, bi in enumerate(b):
        xi, info = spla.bicgstab(C, bi, x0=None if x0 is None else x0[i], rtol=rtol, atol=0.0,
                                 maxiter=20000)
        if info != 0:
            raise RuntimeError("oracle BiCGStab did not converge (info=%d)" % info)
        out.append(xi)
    return np.stack(out), None


def correct(geo: Geometry, h, A, p):
    """u = h - A^-1 grad p (eq. velCorrDiscrete)."""
    return h - geo.grad(p) / A


def face_flux_divergence(geo: Geometry, h, A, p, p_lag, u_b):
    """Net outward corrected face flux per cell, summed face by face:
    lerp(J T_j . h) - P_f (p_F - p_P) - deferred cross flux, plus the Dirichlet flux."""
    N = geo.N
    W = np.einsum("jin,in->jn", geo.JT, h)
    div = np.zeros(N, dtype=np.result_type(h, p))
    cross = None
    if geo.non_orthogonal:
        kap = 1.0 / A
        g = np.stack([geo.Gt[k] @ p_lag for k in range(geo.d)])
    for j in range(geo.d):
        P, F = geo.faces[j]
        pf = 0.5 * (geo.alpha[j, j, P] / A[P] + geo.alpha[j, j, F] / A[F])
        flux = 0.5 * (W[j, P] + W[j, F]) - pf * (p[F] - p[P])
        if geo.non_orthogonal:
            for k in range(geo.d):
                if k != j:
                    w = 0.5 * (geo.alpha[j, k, P] * kap[P] + geo.alpha[j, k, F] * kap[F])
                    flux = flux - w * 0.5 * (g[k, P] + g[k, F])
        np.add.at(div, P, flux)
        np.add.at(div, F, -flux)
    if geo.nb:
        div = div + sum(geo.Bflux[i] @ u_b[i] for i in range(geo.d))
    return div


@dataclass
class StepRecord:
    u_n: np.ndarray
    p_n: np.ndarray
    nu: np.ndarray
    S: np.ndarray
    u_b: np.ndarray
    dt: float
    H: sp.csr_matrix
    A: np.ndarray
    b_u: np.ndarray
    b: np.ndarray
    Pm: sp.csr_matrix
    u_star: np.ndarray
    h1: np.ndarray
    rhs1: np.ndarray
    p1: np.ndarray
    u1: np.ndarray
    h2: np.ndarray
    rhs2: np.ndarray
    p2: np.ndarray
    u2: np.ndarray
    lu: Optional[object] = None
    grad_p_in_predictor: bool = True

    @property
    def u_next(self):
        return self.u2

    @property
    def p_next(self):
        return self.p2


def step(geo: Geometry, u_n, p_n, nu, S, dt, u_b, mode="direct", rtol=1e-13,
         n_correctors=2, grad_p_in_predictor=True) -> StepRecord:
    """One PISO step (App. A.2): predictor and two pressure correctors.

    grad_p_in_predictor keeps -grad p^n on the predictor right-hand side (eqs.
    implEuler1 and advectionMat); without it the predictor uses b_u alone, as the
    discrete eq. velRHSdiscrete is printed.  Steady states do not depend on it, but with
    it the lagged pressure can feed a growing decoupled mode when nu dt / dx^2 >> 1.
    """
    u_n = np.asarray(u_n)
    nu_f = geo.nu_field(nu)
    H, A = assemble_C(geo, u_n, nu_f, dt)
    b_u = predictor_rhs(geo, u_n, nu_f, S, dt, u_b)
    b = b_u - geo.grad(p_n) if grad_p_in_predictor else b_u.copy()
    u_star, lu = solve_velocity(H, A, b, mode, rtol, x0=u_n)
    Pm = pressure_matrix(geo, A)
    hs, rhss, ps, us = [], [], [], []
    u, p_lag = u_star, p_n
    for _ in range(n_correctors):
        h, rhs = h_and_rhs(geo, H, A, b_u, u, u_b, p_lag)
        p = solve_pressure(Pm, rhs, mode, rtol, x0=p_lag)
        u = correct(geo, h, A, p)
        hs.append(h); rhss.append(rhs); ps.append(p); us.append(u)
        p_lag = p
    return StepRecord(u_n, np.asarray(p_n), nu_f, S, u_b, dt, H, A, b_u, b, Pm, u_star,
                      hs[0], rhss[0], ps[0], us[0], hs[-1], rhss[-1], ps[-1], us[-1], lu,
                      grad_p_in_predictor)
