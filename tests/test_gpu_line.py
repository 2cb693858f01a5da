"""Line smoothing on the fine multigrid level (single-block grids stretched along one
axis): which axis the library picks, the step against the oracle's direct solve on
shapes that leave segments and lanes of the line kernels empty, and the iteration count
against point smoothing on the same grid.

The smoother only changes how fast the pressure CG converges, so the step agrees with
the oracle to solver tolerance whichever smoother runs.
"""
import math

import numpy as np
import pytest

import cases
from oracle.adjoint import step_vjp
from oracle.piso import Geometry, step as oracle_step
from tests.gpu_common import dev, host, random_state, rel, rel_p, say, small_cases, tight_opts

pytestmark = pytest.mark.gpu


def _api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api
    return api


def _box(dims, stretch_axis, periodic_axes, beta=2.0, extent=(2 * math.pi, 2 * math.pi, 1.0)):
    """Single block, tanh-stretched along one axis with walls at both of its ends; the
    listed axes wrap onto themselves, the remaining sides are walls."""
    d = len(dims)
    verts = []
    for a in range(d):
        if a == stretch_axis:
            verts.append(cases.tanh_vertices(dims[a], beta, 0.0, extent[a]))
        else:
            verts.append(np.linspace(0.0, extent[a], dims[a] + 1))
    T, J, c = cases.tensor_metrics(verts)
    sides = cases.periodic_sides(0, d, periodic_axes)
    for a in range(d):
        if a not in periodic_axes:
            sides += [cases.Side(0, 2 * a, cases.DIRICHLET), cases.Side(0, 2 * a + 1, cases.DIRICHLET)]
    block = tuple(dims) + ((1,) if d == 2 else ())
    dom = cases.Domain(d, [block], sides, T, J, c)
    N = dom.n_cells
    u_b = cases.boundary_values(dom, lambda si: np.zeros(d))
    rng = np.random.default_rng(21)
    u0 = 0.3 * rng.standard_normal((d, N))
    S = np.zeros((d, N))
    name = "box" + "x".join(str(n) for n in dims)
    return cases.Case(name, dom, u0, np.zeros(N), S, 0.01, 0.02, u_b, 1)


def line_cases():
    return {
        # lines along y of 37 cells (8-cell segments, the last one ragged, three empty),
        # 120 lines: a partly filled last work-group
        "channel40x37x3": (cases.channel(40, 37, 3), 1),
        # lines along z; x wraps, y is walled
        "zbox12x9x16": (_box((12, 9, 16), 2, (0,)), 2),
        # 2D, lines along y of 90 cells (12-cell segments), walls on every side
        "ybox2d20x90": (_box((20, 90), 1, (), extent=(4.0, 1.0)), 1),
        # lines along y of 112 cells: 16-cell segments (the longest kind), the last ragged
        "channel8x112x8": (cases.channel(8, 112, 8), 1),
    }


def test_line_axis_choice(monkeypatch):
    api = _api()
    for name, case in small_cases().items():
        ctx = api.Context(case.domain, "f64")
        want = 1 if name.startswith("channel") else 0
        say("%s: line axis %d" % (name, ctx.mg_line_axis))
        assert ctx.mg_line_axis == want
    for name, (case, axis) in line_cases().items():
        assert api.Context(case.domain, "f64").mg_line_axis == axis, name
    monkeypatch.setenv("PISO_MG_LINE", "0")
    assert api.Context(small_cases()["channel"].domain, "f64").mg_line_axis == 0


@pytest.mark.parametrize("name", list(line_cases()))
def test_line_step_f64(name, monkeypatch):
    """FP64 step with line smoothing: the oracle's direct-solve step to solver tolerance,
    and no more pressure iterations than point smoothing needs on the same grid."""
    api = _api()
    case, axis = line_cases()[name]
    u, p, S, ub, nu = random_state(case, seed=31)
    ref = oracle_step(Geometry(case.domain), u, p, nu, S, case.dt, ub)
    iters = {}
    for line in (True, False):
        if not line:
            monkeypatch.setenv("PISO_MG_LINE", "0")
        ctx = api.Context(case.domain, "f64")
        monkeypatch.delenv("PISO_MG_LINE", raising=False)
        assert ctx.mg_line_axis == (axis if line else 0)
        o = tight_opts(ctx)
        t = ctx.dtype
        u1, p1, info = ctx.step(dev(u, t), dev(p, t), dev(nu, t), dev(S, t), dev(ub, t), case.dt, o, info=True)
        eu, ep = rel(host(u1), ref.u2), rel_p(host(p1), ref.p2)
        iters[line] = [q["iters"] for q in info["pres"]]
        say("%s line %s: iters %s, rel err u %.2e p %.2e" % (name, line, iters[line], eu, ep))
        assert all(q["status"] == 0 for q in info["pres"])
        assert eu < 1e-9 and ep < 1e-8
    assert sum(iters[True]) <= sum(iters[False])


@pytest.mark.parametrize("prec", ["f32", "mixed"])
def test_line_step_single_precision(prec):
    api = _api()
    for name, (case, axis) in line_cases().items():
        u, p, S, ub, nu = random_state(case, seed=32)
        ref = oracle_step(Geometry(case.domain), u, p, nu, S, case.dt, ub)
        ctx = api.Context(case.domain, prec)
        assert ctx.mg_line_axis == axis
        t = ctx.dtype
        u1, p1, info = ctx.step(dev(u, t), dev(p, t), dev(nu, t), dev(S, t), dev(ub, t), case.dt,
                                ctx.default_opts(), info=True)
        eu, ep = rel(host(u1), ref.u2), rel_p(host(p1), ref.p2)
        say("%s %s: iters %s, rel err u %.2e p %.2e" % (name, prec, [q["iters"] for q in info["pres"]], eu, ep))
        # MIXED: FP64-level to its residuals (1e-10 velocity, 1e-8 pressure)
        assert eu < (1e-7 if prec == "mixed" else 1e-5) and ep < (1e-6 if prec == "mixed" else 1e-5)


def test_line_adjoint_matches_point_adjoint(monkeypatch):
    """The adjoint pressure solves run the same preconditioner: the gradient of one FP64
    step agrees with the point-smoothed one to solver tolerance."""
    api = _api()
    case, _ = line_cases()["zbox12x9x16"]
    u, p, S, ub, nu = random_state(case, seed=33)
    rng = np.random.default_rng(34)
    grads = []
    for env in (None, "0"):
        if env:
            monkeypatch.setenv("PISO_MG_LINE", env)
        ctx = api.Context(case.domain, "f64")
        monkeypatch.delenv("PISO_MG_LINE", raising=False)
        t = ctx.dtype
        du1 = dev(rng.standard_normal(u.shape), t) if not grads else grads[0]["_du1"]
        dp1 = dev(rng.standard_normal(p.shape), t) if not grads else grads[0]["_dp1"]
        o = tight_opts(ctx)
        tape = ctx.new_tape()
        args = (dev(u, t), dev(p, t), dev(nu, t), dev(S, t), dev(ub, t))
        ctx.step(*args, case.dt, o, tape=tape)
        g = ctx.step_backward(tape, args[0], args[1], args[2], args[4], case.dt, du1, dp1, o)
        out = {k: host(v) for k, v in g.items()}
        out["_du1"], out["_dp1"] = du1, dp1
        grads.append(out)
    for k in grads[0]:
        if k.startswith("_"):
            continue
        e = rel(grads[0][k], grads[1][k])
        say("grad %s: line vs point rel %.2e" % (k, e))
        assert e < 1e-9


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_line_adjoint_vs_oracle(prec):
    """The adjoint of a step with 3D line smoothing (lines of 96 cells: 12-cell
    segments) against the oracle's step_vjp: F64 <= 1e-8; F32 <= 1e-5, except the
    pressure gradient, which inherits the forward pressure's cancellation in FP32 storage
    (measured 1.5e-5): 1e-4."""
    api = _api()
    case = cases.channel(16, 96, 8)
    u, p, S, ub, nu = random_state(case, seed=35)
    if prec == "f32":
        u, p, S, ub, nu = [np.asarray(x, dtype=np.float32).astype(np.float64) for x in (u, p, S, ub, nu)]
    rng = np.random.default_rng(36)
    w = rng.standard_normal(u.shape)
    wp = rng.standard_normal(p.shape)
    if prec == "f32":
        w, wp = w.astype(np.float32).astype(np.float64), wp.astype(np.float32).astype(np.float64)
    ctx = api.Context(case.domain, prec)
    assert ctx.mg_line_axis == 1
    t = ctx.dtype
    o = tight_opts(ctx) if prec == "f64" else ctx.default_opts()
    tape = ctx.new_tape()
    args = (dev(u, t), dev(p, t), dev(nu, t), dev(S, t), dev(ub, t))
    ctx.step(*args, case.dt, o, tape=tape)
    g = ctx.step_backward(tape, args[0], args[1], args[2], args[4], case.dt, dev(w, t), dev(wp, t), o)
    geo = Geometry(case.domain)
    ref = oracle_step(geo, u, p, nu, S, case.dt, ub)
    gr = step_vjp(geo, ref, w, wp)
    for k, key in (("u", "u_n"), ("p", "p_n"), ("S", "S"), ("nu", "nu"), ("u_b", "u_b")):
        e = rel(host(g[k]), gr[key])
        say("%s grad %s rel %.2e" % (prec, k, e))
        tol = 1e-8 if prec == "f64" else (1e-4 if k == "p" else 1e-5)
        assert e < tol, k
