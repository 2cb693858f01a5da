"""Dense, loop-by-loop PISO step used only to pin the oracle (tiny grids).

Written independently of oracle/: its own neighbour search over the side segments,
its own dense matrices filled cell by cell and face by face following App. A.3 of the
paper (same readings as the oracle), numpy.linalg.solve for the predictor and the
minimum-norm least-squares solution for the singular pressure system.
"""
import numpy as np

from cases import CONNECT, segment_extent


class Mesh:
    def __init__(self, dom):
        self.dom = dom
        self.d = dom.dim
        self.off = [0]
        for nx, ny, nz in dom.blocks:
            self.off.append(self.off[-1] + nx * ny * nz)
        self.N = self.off[-1]
        self.cells = []
        for b, (nx, ny, nz) in enumerate(dom.blocks):
            for k in range(nz):
                for j in range(ny):
                    for i in range(nx):
                        self.cells.append((b, (i, j, k)))
        # Dirichlet face numbering: segments in list order, tangential t0 fastest
        self.bstart = {}
        n = 0
        for si, seg in enumerate(dom.sides):
            if seg.kind != CONNECT:
                (b0, b1), (e0, e1) = segment_extent(dom, seg)
                self.bstart[si] = n
                n += (e0 - b0) * (e1 - b1)
        self.NB = n

    def index(self, b, ijk):
        nx, ny, nz = self.dom.blocks[b]
        i, j, k = ijk
        return self.off[b] + i + nx * (j + ny * k)

    def neighbour(self, P, axis, side):
        """('cell', F) or ('bnd', face index)."""
        b, ijk = self.cells[P]
        n = self.dom.blocks[b]
        q = list(ijk)
        q[axis] += 1 if side == 1 else -1
        if 0 <= q[axis] < n[axis]:
            return ("cell", self.index(b, q))
        tang = [ijk[a] for a in range(3) if a != axis]
        for si, seg in enumerate(self.dom.sides):
            if seg.block != b or seg.side != 2 * axis + side:
                continue
            (b0, b1), (e0, e1) = segment_extent(self.dom, seg)
            t0, t1 = tang[0], tang[1]
            if not (b0 <= t0 < e0 and b1 <= t1 < e1):
                continue
            if seg.kind == CONNECT:
                ob = seg.other_block
                on = self.dom.blocks[ob]
                o = [t0 - b0 + seg.other_begin[0], t1 - b1 + seg.other_begin[1]]
                r = [0, 0, 0]
                others = [a for a in range(3) if a != axis]
                r[others[0]], r[others[1]] = o[0], o[1]
                r[axis] = 0 if side == 1 else on[axis] - 1
                return ("cell", self.index(ob, r))
            return ("bnd", self.bstart[si] + (t0 - b0) + (e0 - b0) * (t1 - b1))
        raise AssertionError("uncovered face")


def brute_step(dom, u_n, p_n, nu, S, dt, u_b):
    m = Mesh(dom)
    d, N = m.d, m.N
    T, J = dom.T, dom.J
    nu = np.broadcast_to(np.asarray(nu, dtype=float), (N,))
    alpha = np.zeros((d, d, N))
    for P in range(N):
        for j in range(d):
            for k in range(d):
                alpha[j, k, P] = J[P] * sum(T[j, i, P] * T[k, i, P] for i in range(d))

    def U(P, j, vel):
        return J[P] * sum(T[j, i, P] * vel[i] for i in range(d))

    def tgrad(field, P, k):
        tp = m.neighbour(P, k, 1)
        tm = m.neighbour(P, k, 0)
        if tp[0] == "cell" and tm[0] == "cell":
            return 0.5 * (field[tp[1]] - field[tm[1]])
        if tp[0] == "cell":
            return field[tp[1]] - field[P]
        if tm[0] == "cell":
            return field[P] - field[tm[1]]
        return 0.0

    def bnd_tgrad(vals, P, j, s, k):
        own = m.neighbour(P, j, s)[1]
        got = []
        for side in (1, 0):
            q = m.neighbour(P, k, side)
            if q[0] == "cell":
                r = m.neighbour(q[1], j, s)
                got.append(r[1] if r[0] == "bnd" else None)
            else:
                got.append(None)
        bp, bm = got
        if bp is not None and bm is not None:
            return 0.5 * (vals[bp] - vals[bm])
        if bp is not None:
            return vals[bp] - vals[own]
        if bm is not None:
            return vals[own] - vals[bm]
        return 0.0

    C = np.zeros((N, N))
    b_u = np.zeros((d, N))
    for P in range(N):
        C[P, P] += 1.0 / dt
        for i in range(d):
            b_u[i, P] += u_n[i, P] / dt + S[i, P]
        for j in range(d):
            for s in (0, 1):
                Nf = 1.0 if s == 1 else -1.0
                kind, F = m.neighbour(P, j, s)
                if kind == "cell":
                    Uf = 0.5 * (U(P, j, u_n[:, P]) + U(F, j, u_n[:, F]))
                    knu = 0.5 * (alpha[j, j, P] * nu[P] + alpha[j, j, F] * nu[F])
                    C[P, F] += (0.5 * Nf * Uf - knu) / J[P]
                    C[P, P] += (0.5 * Nf * Uf + knu) / J[P]
                    for k in range(d):
                        if k == j:
                            continue
                        w = 0.5 * (alpha[j, k, P] * nu[P] + alpha[j, k, F] * nu[F])
                        for i in range(d):
                            t = 0.5 * (tgrad(u_n[i], P, k) + tgrad(u_n[i], F, k))
                            b_u[i, P] += Nf * w * t / J[P]
                else:
                    C[P, P] += 2.0 * alpha[j, j, P] * nu[P] / J[P]
                    ub = u_b[:, F]
                    Ub = U(P, j, ub)
                    for i in range(d):
                        b_u[i, P] += ub[i] * (2.0 * alpha[j, j, P] * nu[P] - Nf * Ub) / J[P]
                    for k in range(d):
                        if k == j:
                            continue
                        for i in range(d):
                            g = bnd_tgrad(u_b[i], P, j, s, k)
                            b_u[i, P] += Nf * alpha[j, k, P] * nu[P] * g / J[P]

    def gradp(p):
        g = np.zeros((d, N))
        for P in range(N):
            for j in range(d):
                kp, Fp = m.neighbour(P, j, 1)
                km, Fm = m.neighbour(P, j, 0)
                pp = p[Fp] if kp == "cell" else p[P]
                pm = p[Fm] if km == "cell" else p[P]
                for i in range(d):
                    g[i, P] += T[j, i, P] * (pp - pm) / 2.0
        return g

    b = b_u - gradp(p_n)
    u_star = np.stack([np.linalg.solve(C, b[i]) for i in range(d)])
    A = np.diag(C).copy()
    Hm = C - np.diag(A)
    Pm = np.zeros((N, N))
    for P in range(N):
        for j in range(d):
            for s in (0, 1):
                kind, F = m.neighbour(P, j, s)
                if kind == "cell":
                    pf = 0.5 * (alpha[j, j, P] / A[P] + alpha[j, j, F] / A[F])
                    Pm[P, F] += pf
                    Pm[P, P] -= pf

    def corrector(u, p_lag):
        h = np.stack([(b_u[i] - Hm @ u[i]) / A for i in range(d)])
        rhs = np.zeros(N)
        for P in range(N):
            for j in range(d):
                for s in (0, 1):
                    Nf = 1.0 if s == 1 else -1.0
                    kind, F = m.neighbour(P, j, s)
                    if kind == "cell":
                        rhs[P] += Nf * 0.5 * (U(P, j, h[:, P]) + U(F, j, h[:, F]))
                        for k in range(d):
                            if k == j:
                                continue
                            w = 0.5 * (alpha[j, k, P] / A[P] + alpha[j, k, F] / A[F])
                            t = 0.5 * (tgrad(p_lag, P, k) + tgrad(p_lag, F, k))
                            rhs[P] -= Nf * w * t
                    else:
                        rhs[P] += Nf * U(P, j, u_b[:, F])
        rhs = rhs - rhs.mean()
        p = np.linalg.lstsq(Pm, rhs, rcond=None)[0]
        u = h - gradp(p) / A
        return h, p, u

    h1, p1, u1 = corrector(u_star, p_n)
    h2, p2, u2 = corrector(u1, p1)
    return dict(A=A, C=C, Pm=Pm, b_u=b_u, u_star=u_star, h1=h1, p1=p1, u1=u1, h2=h2, p2=p2, u2=u2)
