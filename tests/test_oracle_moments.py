"""Pins of the arbitrary-order moments and budget-term oracle (Sec. 2.5; formulas in
oracle/moments.py): the definitions on pooled samples by plain loops, order
independence, the covariance oracle at order 2, complex-step gradients, the field
gradient on fields it differentiates exactly, the profile operators against the step's
own diffusion matrix, and the budget terms against a brute-force evaluation from the
pooled samples."""
import numpy as np
import pytest
import scipy.sparse as sp

import cases
from oracle import moments as om
from oracle import stats as ost
from oracle.piso import Geometry, assemble_C


def _fields(rng, dims, m, n, offset=0.0):
    N = dims[0] * dims[1] * dims[2]
    return [offset + rng.standard_normal((m, N)) * (1 + 0.3 * q) for q in range(n)]


def _pooled(us, dims, axis, p):
    nx, ny, nz = dims
    out = []
    for u in us:
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    if (i, j, k)[axis] == p:
                        out.append(u[:, i + nx * (j + ny * k)])
    return np.array(out)


@pytest.mark.parametrize("dims,m,K,axis", [((5, 4, 3), 3, 4, 1), ((4, 3, 5), 3, 3, 2), ((6, 5, 1), 2, 4, 1),
                                           ((3, 4, 2), 6, 2, 0)])
def test_online_equals_pooled_definition(dims, m, K, axis):
    rng = np.random.default_rng(0)
    us = _fields(rng, dims, m, 4, offset=2.0)
    st = om.empty_state(dims[axis], m, K)
    for u in us:
        st = om.accumulate(st, u, dims, axis)
    mean, mom = om.finalize(st)
    idx = om.multi_indices(m, K)
    for p in range(dims[axis]):
        X = _pooled(us, dims, axis, p)
        mu = X.mean(axis=0)
        assert np.allclose(mean[p], mu, rtol=1e-13, atol=1e-13)
        for q, t in enumerate(idx):
            ref = np.mean(np.prod([X[:, i] - mu[i] for i in t], axis=0))
            assert abs(mom[p, q] - ref) <= 1e-11 * max(1.0, abs(ref)), (p, t)


def test_order_independence_and_order2_is_covariance():
    rng = np.random.default_rng(1)
    dims, m = (6, 4, 3), 3
    us = _fields(rng, dims, m, 5, offset=-1.0)
    a, b = om.empty_state(4, m, 4), om.empty_state(4, m, 4)
    c = ost.empty_state(4, m)
    for u in us:
        a = om.accumulate(a, u, dims, 1)
        c = ost.accumulate(c, u, dims, 1)
    for u in us[::-1]:
        b = om.accumulate(b, u, dims, 1)
    assert np.allclose(a["S"], b["S"], rtol=1e-11, atol=1e-11)
    _, cov = ost.finalize(c)
    _, mom = om.finalize(a)
    assert np.allclose(mom[:, :6], cov, rtol=1e-12, atol=1e-13)
    # a constant field has zero central moments of every order
    z = om.empty_state(4, m, 4)
    for _ in range(3):
        z = om.accumulate(z, np.full((m, 72), 1.5), dims, 1)
    assert np.all(z["S"] == 0.0)


@pytest.mark.parametrize("m,K", [(3, 4), (6, 2), (2, 3)])
def test_vjp_complex_step(m, K):
    rng = np.random.default_rng(2)
    dims, axis = (4, 5, 3), 1
    us = _fields(rng, dims, m, 3, offset=0.5)
    np_ = dims[axis]
    nq = len(om.multi_indices(m, K))
    mbar = rng.standard_normal((np_, m))
    obar = rng.standard_normal((np_, nq))

    def loss(fields):
        st = om.empty_state(np_, m, K)
        for u in fields:
            st = om.accumulate(st, u, dims, axis)
        mu, mo = om.finalize(st)
        return np.sum(mbar * mu) + np.sum(obar * mo)

    st = om.empty_state(np_, m, K)
    for u in us:
        st = om.accumulate(st, u, dims, axis)
    for q in range(3):
        g = om.moments_vjp(st, us[q], dims, axis, mbar, obar)
        v = rng.standard_normal(us[q].shape)
        h = 1e-30
        pert = [u.astype(complex) for u in us]
        pert[q] = pert[q] + 1j * h * v
        cs = loss(pert).imag / h
        assert abs(cs - np.sum(g * v)) <= 1e-11 * max(1.0, abs(cs))


def _box(nx, ny, nz, Ly=1.0, beta=None):
    """Periodic x, z; walls in y (uniform, or tanh-stretched with beta)."""
    xv = np.linspace(0.0, 2 * np.pi, nx + 1)
    yv = np.linspace(0.0, Ly, ny + 1) if beta is None else cases.tanh_vertices(ny, beta, 0.0, Ly)
    zv = np.linspace(0.0, np.pi, nz + 1)
    T, J, c = cases.tensor_metrics([xv, yv, zv])
    sides = cases.periodic_sides(0, 3, (0, 2)) + [cases.Side(0, 2, cases.DIRICHLET), cases.Side(0, 3, cases.DIRICHLET)]
    return cases.Domain(3, [(nx, ny, nz)], sides, T, J, c), c


def test_field_gradient_exact_cases():
    """On a uniform grid, central differences with the ghost reading are exact for fields
    linear in y (walls carrying the field's face values) and give the closed-form symbol
    sin(k h)/h for a periodic mode in x; with phi_b = None the wall face takes the cell's
    value."""
    nx, ny, nz = 8, 6, 4
    dom, c = _box(nx, ny, nz)
    geo = Geometry(dom)
    x, y, z = c
    a = np.array([2.0, -1.0, 0.5])
    phi = np.stack([a[q] * y + 3.0 for q in range(3)])
    yb = np.where(geo.bs == 1, 1.0, 0.0)         # wall faces at y = 0 and y = 1
    phi_b = np.stack([a[q] * yb + 3.0 for q in range(3)])
    g = om.field_gradient(geo, phi, phi_b)
    assert np.allclose(g[1], a[:, None], rtol=1e-12, atol=1e-12)
    assert np.allclose(g[0], 0.0, atol=1e-12) and np.allclose(g[2], 0.0, atol=1e-12)
    h = 2 * np.pi / nx
    s = np.sin(2 * x)[None]
    gs = om.field_gradient(geo, s, np.zeros((1, geo.nb)))
    assert np.allclose(gs[0, 0], 2 * np.cos(2 * x) * np.sin(2 * h) / (2 * h), rtol=1e-12, atol=1e-12)
    # pressure reading: p_b = p_P, so the wall cell's difference is one-sided over half
    gp = om.field_gradient(geo, phi[:1], None)
    P0 = 0  # a first-row cell: (p(y1) - p(y0)) / 2 * T_yy
    assert np.isclose(gp[1, 0, P0], 0.5 * (phi[0, nx] - phi[0, 0]) * geo.T[1, 1, P0])


def test_profile_operators_match_step_diffusion():
    """D = d^2/dy^2 across the planes equals minus the step's own diffusion operator
    (eq. difMatDiscrete with nu = 1, no advection, 1/dt -> 0) applied to a field that is
    constant over each plane; the first derivative is exact for linear profiles through
    the wall values."""
    nx, ny, nz = 4, 9, 2
    dom, c = _box(nx, ny, nz, beta=1.5)
    geo = Geometry(dom)
    rng = np.random.default_rng(3)
    f = rng.standard_normal(ny)
    T, J = om._plane_metric(geo, (nx, ny, nz), 1)
    d2 = om.profile_d2(f, T, J, (0.0, 0.0), periodic=False)
    H, A = assemble_C(geo, np.zeros((3, geo.N)), np.ones(geo.N), 1e300)
    C = H + sp.diags(A)
    field = np.repeat(np.repeat(f[None, :, None], nx, axis=2), nz, axis=0).reshape(-1)
    ref = -(C @ field).reshape(nz, ny, nx)[0, :, 0]
    assert np.allclose(d2, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # the first derivative: exact for a linear profile on a uniform grid
    dom_u, cu = _box(nx, ny, nz)
    geo_u = Geometry(dom_u)
    Tu, Ju = om._plane_metric(geo_u, (nx, ny, nz), 1)
    yu = cu[1].reshape(nz, ny, nx)[0, :, 0]
    assert np.allclose(om.profile_d1(2.0 * yu - 0.5, Tu, (-0.5, 1.5), False), 2.0, rtol=1e-12)


def test_budget_against_pooled_brute_force():
    """Every budget term from the online statistics equals the same term computed by
    loops over the pooled samples of each plane (means, products of deviations) and the
    profile operators."""
    nx, ny, nz = 6, 5, 4
    dom, c = _box(nx, ny, nz, beta=1.2)
    geo = Geometry(dom)
    dims = (nx, ny, nz)
    rng = np.random.default_rng(4)
    steps = 3
    us = [rng.standard_normal((3, geo.N)) + np.array([[1.0], [0.2], [-0.1]]) for _ in range(steps)]
    ps = [rng.standard_normal(geo.N) for _ in range(steps)]
    ub = rng.standard_normal((3, geo.nb)) * 0.0
    su = om.empty_state(ny, 3, 3)
    sg = [om.empty_state(ny, 3, 2) for _ in range(3)]
    sup = om.empty_state(ny, 6, 2)
    grads, gps = [], []
    for u, p in zip(us, ps):
        g = om.field_gradient(geo, u, ub)
        gp = om.field_gradient(geo, p[None], None)[:, 0]
        grads.append(g)
        gps.append(gp)
        su = om.accumulate(su, u, dims, 1)
        for k in range(3):
            sg[k] = om.accumulate(sg[k], g[k], dims, 1)
        sup = om.accumulate(sup, np.concatenate([u, gp]), dims, 1)
    out = om.budget(geo, dims, 1, om.finalize(su), [om.finalize(s)[1] for s in sg], om.finalize(sup)[1],
                    (np.zeros(3), np.zeros(3)))
    # brute force
    T, J = om._plane_metric(geo, dims, 1)
    U = np.zeros((ny, 3))
    R = np.zeros((ny, 3, 3))
    T3 = np.zeros((ny, 3, 3))
    eps = np.zeros((ny, 3, 3))
    Pi = np.zeros((ny, 3, 3))
    for pl in range(ny):
        X = _pooled(us, dims, 1, pl)
        G = [_pooled([g[k] for g in grads], dims, 1, pl) for k in range(3)]
        Gp = _pooled(gps, dims, 1, pl)
        U[pl] = X.mean(axis=0)
        dX = X - U[pl]
        for i in range(3):
            for j in range(3):
                R[pl, i, j] = np.mean(dX[:, i] * dX[:, j])
                T3[pl, i, j] = np.mean(dX[:, i] * dX[:, j] * dX[:, 1])
                eps[pl, i, j] = 2 * sum(np.mean((G[k][:, i] - G[k][:, i].mean()) * (G[k][:, j] - G[k][:, j].mean()))
                                        for k in range(3))
                Pi[pl, i, j] = -(np.mean(dX[:, i] * (Gp[:, j] - Gp[:, j].mean()))
                                 + np.mean(dX[:, j] * (Gp[:, i] - Gp[:, i].mean())))
    dU = np.stack([om.profile_d1(U[:, i], T, (0.0, 0.0), False) for i in range(3)], axis=1)
    for q, (i, j) in enumerate([(i, j) for i in range(3) for j in range(i, 3)]):
        P = -(R[:, i, 1] * dU[:, j] + R[:, j, 1] * dU[:, i])
        Tt = -om.profile_d1(T3[:, i, j], T, (0.0, 0.0), False)
        D = om.profile_d2(R[:, i, j], T, J, (0.0, 0.0), False)
        for name, ref in (("P", P), ("eps", eps[:, i, j]), ("T", Tt), ("D", D), ("Pi", Pi[:, i, j])):
            assert np.allclose(out[name][:, q], ref, rtol=1e-10, atol=1e-10 * max(1.0, np.abs(ref).max())), (name, i, j)
