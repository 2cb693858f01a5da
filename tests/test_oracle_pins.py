"""Pins of the FP64 oracle against things other than itself (no GPU).

* dense loop-by-loop brute force on tiny grids (single/multi-block, 2D/3D, sheared);
* plane Poiseuille closed form (App. B.1: u = G/(2 nu) y(1-y), u_max = 0.125);
* Taylor-Green linear-regime decay factor and continuum decay exp(-2 nu t);
* exact Fourier symbols of a full linearised step on a sheared periodic grid
  (pins the signs and weights of the deferred non-orthogonal terms);
* zero face-flux divergence after each correction; invariants (symmetry and
  semi-definiteness of P, uniform flow, 90-degree rotation of the cavity, axis swap);
* topology validation errors.
"""
import math
import os

import numpy as np
import pytest

import cases
from oracle.piso import Geometry, face_flux_divergence, pressure_matrix, step
from oracle.topology import TopologyError, build_topology
from tests.bruteforce import brute_step

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _random_state(case, seed):
    rng = np.random.default_rng(seed)
    d, N = case.u0.shape
    u = case.u0 + 0.2 * rng.standard_normal((d, N))
    p = rng.standard_normal(N)
    S = rng.standard_normal((d, N))
    ub = case.u_b + 0.1 * rng.standard_normal(case.u_b.shape)
    nu = case.nu * (1.0 + 0.2 * rng.random(N))
    return u, p, S, ub, nu


def _two_block():
    """Two 3x4 blocks side by side along x, periodic in x through the pair, walls in y."""
    xv = np.linspace(0, 1, 4)
    yv = np.array([0.0, 0.2, 0.45, 0.75, 1.0])
    T0, J0, c0 = cases.tensor_metrics([xv, yv])
    T1, J1, c1 = cases.tensor_metrics([xv + 1.0, yv])
    T, J, c = cases.concat_blocks([(T0, J0, c0), (T1, J1, c1)])
    S_ = cases.Side
    sides = [S_(0, 1, cases.CONNECT, other_block=1), S_(1, 0, cases.CONNECT, other_block=0),
             S_(1, 1, cases.CONNECT, other_block=0), S_(0, 0, cases.CONNECT, other_block=1),
             S_(0, 2, cases.DIRICHLET), S_(0, 3, cases.DIRICHLET),
             S_(1, 2, cases.DIRICHLET), S_(1, 3, cases.DIRICHLET)]
    dom = cases.Domain(2, [(3, 4, 1), (3, 4, 1)], sides, T, J, c)
    ub = cases.boundary_values(dom, lambda si: np.array([0.7, 0.0]) if dom.sides[si].side == 3
                               else np.zeros(2))
    return cases.Case("two_block", dom, np.zeros((2, 24)), np.zeros(24), np.zeros((2, 24)),
                      0.05, 0.1, ub, 1)


def _small_cases():
    return [
        cases.taylor_green(4, dt=0.3),
        cases.lid_cavity(5, n_steps=1),
        cases.channel(4, 3, 3),
        _two_block(),
        cases.sheared_channel(4, 5, shear=0.7),
        cases.cylinder_oh(8, 3, 3),
    ]


@pytest.mark.parametrize("idx", range(6))
def test_bruteforce_dense(idx):
    case = _small_cases()[idx]
    u, p, S, ub, nu = _random_state(case, 10 + idx)
    geo = Geometry(case.domain)
    rec = step(geo, u, p, nu, S, case.dt, ub)
    ref = brute_step(case.domain, u, p, nu, S, case.dt, ub)
    assert _rel(rec.A, ref["A"]) < 1e-13
    assert _rel(rec.b_u, ref["b_u"]) < 1e-13
    assert _rel(rec.Pm.toarray(), ref["Pm"]) < 1e-13
    for name in ("u_star", "h1", "p1", "u1", "h2", "p2", "u2"):
        assert _rel(getattr(rec, name), ref[name]) < 1e-11, name


def _steady(case, n_steps=6, grad_p_in_predictor=False):
    """March to the steady state with a huge dt (nu dt / dy^2 >> 1, so the lagged
    pressure gradient is left out of the predictor; steady states do not depend on it)."""
    geo = Geometry(case.domain)
    u, p = case.u0, case.p0
    for _ in range(n_steps):
        rec = step(geo, u, p, case.nu, case.S, case.dt, case.u_b,
                   grad_p_in_predictor=grad_p_in_predictor)
        u, p = rec.u2, rec.p2
    return geo, u, p


@pytest.mark.parametrize("ny", [8, 32, 100])
def test_poiseuille_closed_form(ny):
    """Uniform grid: the discrete steady state is G/(2nu)(y(1-y) + dy^2/4) exactly."""
    case = cases.poiseuille(4, ny)
    geo, u, p = _steady(case)
    y = case.domain.centres[1]
    dy = 1.0 / ny
    exact = 1.0 / 2.0 * (y * (1 - y) + dy * dy / 4)
    assert np.max(np.abs(u[0] - exact)) < 1e-12
    assert np.max(np.abs(u[1])) < 1e-12
    # the analytic profile itself is met to within G dy^2/(8 nu)
    assert np.max(np.abs(u[0] - 0.5 * y * (1 - y))) <= dy * dy / 8 + 1e-12


def test_poiseuille_steady_with_lagged_pressure():
    case = cases.poiseuille(4, 8)
    geo, u, p = _steady(case, 6, grad_p_in_predictor=True)
    y = case.domain.centres[1]
    exact = 0.5 * (y * (1 - y) + (1.0 / 8) ** 2 / 4)
    assert np.max(np.abs(u[0] - exact)) < 1e-12


def test_poiseuille_golden_umax():
    """The paper's printed maximum velocity for nu = G = 1 on [0, 1]."""
    with open(os.path.join(GOLDEN, "poiseuille_umax.txt")) as f:
        vals = [float(line.split("=")[1]) for line in f if line.startswith("u_max")]
    case = cases.poiseuille(4, 16)
    _, u, _ = _steady(case)
    assert abs(u[0].max() - vals[0]) < 1e-12


def test_poiseuille_stretched_matches_1d_solve():
    """Refined grid: compare with the same finite-volume balance solved as a 1D
    tridiagonal system (flux between cell centres with face conductance equal to the
    mean of the two cells' 1/width, half-cell wall distance)."""
    yv = cases.tanh_vertices(24, 1.7, 0.0, 1.0)
    case = cases.poiseuille(3, vertices_y=yv)
    geo, u, p = _steady(case, 8)
    w = np.diff(yv)
    n = len(w)
    M = np.zeros((n, n))
    for i in range(n):
        for jn in (i - 1, i + 1):
            if 0 <= jn < n:
                g = 0.5 * (1.0 / w[i] + 1.0 / w[jn])
                M[i, i] += g
                M[i, jn] -= g
            else:
                M[i, i] += 2.0 / w[i]
    ref = np.linalg.solve(M, w)          # G * cell width on the right
    prof = u[0].reshape(n, 3)[:, 0]
    assert np.max(np.abs(prof - ref)) < 1e-12


def test_sheared_channel_matches_closed_form():
    """Poiseuille flow on a skewed periodic grid: deferred cross terms must cancel and
    the uniform-grid closed form must be reproduced."""
    case = cases.sheared_channel(6, 8, shear=0.6)
    geo, u, p = _steady(case, 8)
    assert geo.non_orthogonal
    y = case.domain.centres[1]
    dy = 1.0 / 8
    exact = 0.5 * (y * (1 - y) + dy * dy / 4)
    assert np.max(np.abs(u[0] - exact)) < 1e-12
    assert np.max(np.abs(u[1])) < 1e-12


def test_tgv_linear_decay_factor():
    """Amplitude 1e-10: the TGV field is an eigenvector of the compact diffusion with zero
    discrete divergence, so each step multiplies it by 1/(1 + nu dt lambda_h)."""
    n, nu, dt, steps = 32, 0.01, 0.01, 20
    case = cases.taylor_green(n, nu=nu, dt=dt, amplitude=1e-10)
    geo = Geometry(case.domain)
    u, p = case.u0, np.zeros(geo.N)
    for _ in range(steps):
        rec = step(geo, u, p, nu, case.S, dt, case.u_b)
        u, p = rec.u2, rec.p2
    h = 2 * math.pi / n
    lam = 2 * (2 - 2 * math.cos(h)) / h ** 2
    g = 1.0 / (1.0 + nu * dt * lam)
    assert _rel(u, g ** steps * case.u0) < 1e-9
    assert abs(g ** steps - 0.996021) < 1e-6


def test_tgv_full_amplitude_decay():
    """Full amplitude: velocity decays like exp(-2 nu t), pressure like exp(-4 nu t)."""
    rows = []
    for n in (16, 32):
        case = cases.taylor_green(n)
        geo = Geometry(case.domain)
        u, p = case.u0, case.p0
        for _ in range(case.n_steps):
            rec = step(geo, u, p, case.nu, case.S, case.dt, case.u_b)
            u, p = rec.u2, rec.p2
        t = case.n_steps * case.dt
        a = np.sum(u * case.u0) / np.sum(case.u0 * case.u0)
        shape = np.linalg.norm(u - a * case.u0) / np.linalg.norm(u)
        p_err = _rel(p - p.mean(), case.p0 * math.exp(-4 * case.nu * t))
        rows.append((abs(a - math.exp(-2 * case.nu * t)), shape, p_err))
    assert rows[1][0] < 1e-3 and rows[1][1] < 1e-3 and rows[1][2] < 2e-2
    assert rows[1][0] < rows[0][0] and rows[1][1] < rows[0][1] and rows[1][2] < rows[0][2]


@pytest.mark.parametrize("shear", [0.0, 0.5, 1.0])
def test_fourier_symbol_sheared_grid(shear):
    """Single Fourier mode on an affine periodic grid, amplitude 1e-12 (advection is
    negligible): every operator of the step is a multiplication by its symbol, so the
    whole step (predictor, both correctors, lagged cross terms) is known exactly."""
    n, nu, dt = 12, 1.0, 0.05
    dom = cases.sheared_periodic(n, shear)
    geo = Geometry(dom)
    T, J = dom.T[:, :, 0], dom.J[0]
    al = J * T @ T.T
    theta = np.array([2 * math.pi * 1 / n, 2 * math.pi * 2 / n])
    idx = np.arange(n * n)
    xi = np.stack([idx % n, idx // n]).astype(float)
    ph = np.exp(1j * (theta @ xi))
    eps = 1e-12
    uh = eps * np.array([1.0 + 0.3j, -0.4 + 0.8j])
    ph_n = eps * (0.2 - 0.5j)
    u_n = uh[:, None] * ph[None]
    p_n = ph_n * ph
    sn, cs = np.sin(theta), np.cos(theta)
    orth = sum(al[j, j] * (2 * cs[j] - 2) for j in range(2))
    cross = -2 * al[0, 1] * sn[0] * sn[1]
    gam = np.array([sum(T[j, i] * 1j * sn[j] for j in range(2)) for i in range(2)])
    A = 1 / dt + nu * sum(2 * al[j, j] for j in range(2)) / J
    csym = 1 / dt - nu * orth / J
    Hs = csym - A
    b_u = uh / dt + nu * cross / J * uh
    ustar = (b_u - gam * ph_n) / csym
    pis = orth / A

    def corr(u_in, p_lag):
        hh = (b_u - Hs * u_in) / A
        rhs = J * np.sum(gam * hh) - (cross / A) * p_lag
        pp = rhs / pis
        return hh - gam * pp / A, pp

    u1, p1 = corr(ustar, ph_n)
    u2, p2 = corr(u1, p1)
    rec = step(geo, u_n, p_n, nu, np.zeros((2, n * n)), dt, np.zeros((2, 0)))
    assert _rel(rec.u_star, ustar[:, None] * ph) < 1e-9
    assert _rel(rec.p1, p1 * ph) < 1e-9
    assert _rel(rec.u2, u2[:, None] * ph) < 1e-9
    assert _rel(rec.p2, p2 * ph) < 1e-9
    # the symbol of the full (orthogonal + cross) operator, divided by J, tends to the
    # continuum Laplacian symbol -|k|^2 with k = T^T theta (fixes the cross-term sign)
    th = theta * 1e-3
    full = sum(al[j, j] * (2 * np.cos(th[j]) - 2) for j in range(2)) \
        - 2 * al[0, 1] * np.sin(th[0]) * np.sin(th[1])
    k = T.T @ th
    assert abs(full / J + k @ k) / (k @ k) < 1e-5


@pytest.mark.parametrize("mk", [lambda: cases.taylor_green(16), lambda: cases.lid_cavity(16),
                                lambda: cases.channel(6, 8, 6), lambda: cases.sheared_channel(6, 8)])
def test_divergence_after_correction(mk):
    case = mk()
    geo = Geometry(case.domain)
    rec = step(geo, case.u0 + 0.05 * np.random.default_rng(1).standard_normal(case.u0.shape),
               case.p0, case.nu, case.S, case.dt, case.u_b)
    for h, p, pl, rhs in ((rec.h1, rec.p1, rec.p_n, rec.rhs1), (rec.h2, rec.p2, rec.p1, rec.rhs2)):
        assert abs(rhs.sum()) < 1e-9 * np.abs(rhs).sum()         # compatible data
        div = face_flux_divergence(geo, h, rec.A, p, pl, case.u_b)
        assert np.max(np.abs(div)) < 1e-10


def test_pressure_matrix_invariants():
    case = cases.cylinder_oh(8, 3, 3)
    geo = Geometry(case.domain)
    rng = np.random.default_rng(3)
    A = 10.0 + rng.random(geo.N)
    P = pressure_matrix(geo, A).toarray()
    assert np.array_equal(P, P.T)
    ev = np.linalg.eigvalsh(P)
    assert ev.max() < 1e-10 * abs(ev.min())
    assert np.sum(np.abs(ev) < 1e-10 * abs(ev.min())) == 1


def test_uniform_flow_preserved():
    case = cases.taylor_green(8)
    geo = Geometry(case.domain)
    u = np.stack([np.full(geo.N, 0.7), np.full(geo.N, -0.3)])
    rec = step(geo, u, np.zeros(geo.N), 0.01, case.S, 0.1, case.u_b)
    assert np.max(np.abs(rec.u2 - u)) < 1e-14
    assert np.max(np.abs(rec.p2)) < 1e-14


def test_cavity_rotation_equivariance():
    """Rotating the cavity by 90 degrees together with its lid rotates the results."""
    n = 6
    c = cases.lid_cavity(n, beta=1e-6, n_steps=1)
    dom = c.domain
    rng = np.random.default_rng(5)
    u = 0.3 * rng.standard_normal((2, n * n))
    p = rng.standard_normal(n * n)
    geo = Geometry(dom)
    lid = np.array([1.0, 0.0])
    ub = cases.boundary_values(dom, lambda si: lid if dom.sides[si].side == 3 else np.zeros(2))
    rec = step(geo, u, p, c.nu * 50, np.zeros_like(u), c.dt, ub)
    # rotation (x, y) -> (-y, x) about the centre: cell (i, j) -> (n-1-j, i)
    perm = np.zeros(n * n, dtype=int)
    for j in range(n):
        for i in range(n):
            perm[(n - 1 - j) + n * i] = i + n * j
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    u_r = R @ u[:, perm]
    lid_r = R @ lid
    ub_r = cases.boundary_values(dom, lambda si: lid_r if dom.sides[si].side == 0 else np.zeros(2))
    rec_r = step(geo, u_r, p[perm], c.nu * 50, np.zeros_like(u), c.dt, ub_r)
    assert _rel(rec_r.u2, R @ rec.u2[:, perm]) < 1e-12
    assert _rel(rec_r.p2, rec.p2[perm]) < 1e-12


def test_channel_axis_swap():
    """Swapping the two periodic directions of a cubic channel permutes the outputs."""
    c = cases.channel(5, 4, 5)
    geo = Geometry(c.domain)
    rng = np.random.default_rng(7)
    u = c.u0 + rng.standard_normal(c.u0.shape)
    # domain with x and z lengths equal: rebuild with pi in both
    xv = np.linspace(0, math.pi, 6)
    yv = cases.tanh_vertices(4, 1.5, -1, 1)
    T, J, cc = cases.tensor_metrics([xv, yv, xv])
    dom = cases.Domain(3, [(5, 4, 5)], c.domain.sides, T, J, cc)
    geo = Geometry(dom)
    S = rng.standard_normal(u.shape)
    rec = step(geo, u, np.zeros(geo.N), c.nu, S, c.dt, c.u_b)
    idx = np.arange(geo.N)
    i, j, k = idx % 5, (idx // 5) % 4, idx // 20
    perm = k + 5 * (j + 4 * i)
    sw = [2, 1, 0]
    rec_s = step(geo, u[sw][:, perm], np.zeros(geo.N), c.nu, S[sw][:, perm], c.dt, c.u_b)
    assert _rel(rec_s.u2, rec.u2[sw][:, perm]) < 1e-12
    assert _rel(rec_s.p2, rec.p2[perm]) < 1e-12


def test_iterative_matches_direct():
    case = cases.channel(6, 8, 6)
    geo = Geometry(case.domain)
    a = step(geo, case.u0, case.p0, case.nu, case.S, case.dt, case.u_b, mode="direct")
    b = step(geo, case.u0, case.p0, case.nu, case.S, case.dt, case.u_b, mode="iterative")
    assert _rel(b.u2, a.u2) < 1e-11
    assert _rel(b.p2, a.p2) < 1e-9


def test_topology_errors():
    c = cases.lid_cavity(4, n_steps=1)
    dom = c.domain
    bad = cases.Domain(2, dom.blocks, dom.sides[:3], dom.T, dom.J)
    with pytest.raises(TopologyError):
        build_topology(bad)
    twice = cases.Domain(2, dom.blocks, dom.sides + [cases.Side(0, 0, cases.DIRICHLET)], dom.T, dom.J)
    with pytest.raises(TopologyError):
        build_topology(twice)
    # non-conformal: 3x4 block connected to a 3x5 block
    T0, J0, c0 = cases.tensor_metrics([np.linspace(0, 1, 4), np.linspace(0, 1, 5)])
    T1, J1, c1 = cases.tensor_metrics([np.linspace(1, 2, 4), np.linspace(0, 1, 6)])
    T, J, cc = cases.concat_blocks([(T0, J0, c0), (T1, J1, c1)])
    S_ = cases.Side
    sides = [S_(0, 1, cases.CONNECT, other_block=1), S_(1, 0, cases.CONNECT, other_block=0),
             S_(0, 0, cases.DIRICHLET), S_(1, 1, cases.DIRICHLET)] + \
        [S_(b, s, cases.DIRICHLET) for b in (0, 1) for s in (2, 3)]
    with pytest.raises(TopologyError):
        build_topology(cases.Domain(2, [(3, 4, 1), (3, 5, 1)], sides, T, J, cc))
    negJ = cases.Domain(2, dom.blocks, dom.sides, dom.T, -dom.J)
    with pytest.raises(TopologyError):
        build_topology(negJ)
