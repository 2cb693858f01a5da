"""The fine-grained calls of the C-ABI and their backward twins (App. A.5: one adjoint per
forward operation), chained by hand into one PISO step and its adjoint.

Forward: piso_assemble, piso_solve_velocity, then per corrector piso_solve_pressure and
piso_correct, against the oracle's step record.  Backward, in reverse order:
piso_correct_backward, piso_solve_pressure_backward (corrector 2, then 1),
piso_solve_velocity_backward, piso_assemble_backward.  Every intermediate gradient is
compared with the oracle's corresponding adjoint piece (correct_vjp, pressure_solve_vjp,
h_rhs_vjp) and the end results with the oracle's step_vjp and with piso_step_backward.
FP64 with tight solves: relative L2 <= 1e-8 per field and a per-element bound of 1e-8 of
the field's largest magnitude.
"""
import numpy as np
import pytest
import torch

from oracle.adjoint import _Grads, correct_vjp, h_rhs_vjp, pressure_solve_vjp, step_vjp
from oracle.piso import Geometry, step as oracle_step
from tests.gpu_common import dev, host, random_state, rel, rel_p, say, small_cases, tight_opts

pytestmark = pytest.mark.gpu

TOL = 1e-8


def _close(name, gpu, ref, tol=TOL):
    a, b = host(gpu) if torch.is_tensor(gpu) else np.asarray(gpu), np.asarray(ref)
    e = rel(a, b)
    scale = max(float(np.abs(b).max()), 1e-300)
    m = float(np.abs(a - b).max()) / scale
    say("  %-14s rel L2 %.2e  max elem %.2e" % (name, e, m))
    assert e <= tol and m <= tol, name


def _oracle_dC(geo, G):
    d, N = geo.d, geo.N
    out = np.zeros((2, d, N))
    for j in range(d):
        P, _ = geo.faces[j]
        out[0, j, P] = G.Hpf[j]
        out[1, j, P] = G.Hfp[j]
    return out


@pytest.mark.parametrize("name", ["channel_q", "cylinder_q", "sheared", "two_block"])
def test_backward_twins_chain(name):
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api
    say("test_backward_twins_chain", name)
    case = small_cases()[name]
    geo = Geometry(case.domain)
    u, p, S, ub, nu = random_state(case, seed=21)
    rng = np.random.default_rng(22)
    w = rng.standard_normal(u.shape)
    pbar = rng.standard_normal(p.shape)
    dt = case.dt
    rec = oracle_step(geo, u, p, nu, S, dt, ub)

    ctx = api.Context(case.domain, "f64")
    t = ctx.dtype
    o = tight_opts(ctx, 1e-13, 1e-13)
    o.adjoint_warm_start = 0
    ud, pd, Sd, ubd, nud, wd, pbd = (dev(x, t) for x in (u, p, S, ub, nu, w, pbar))
    d, N = ctx.dim, ctx.N

    # ---- forward through the fine-grained calls
    sys = ctx.new_system()
    ctx.assemble(sys, ud, pd, nud, Sd, ubd, dt)
    us = ud.clone()
    ctx.solve_velocity(sys, us, o.vel)
    p1 = pd.clone()
    ctx.solve_pressure(sys, us, ubd, pd, p1, o.pres)
    h1 = sys["h"].clone()
    u1 = ctx.zeros(d, N)
    ctx.correct(sys, p1, pd, ubd, u1)
    p2 = p1.clone()
    ctx.solve_pressure(sys, u1, ubd, p1, p2, o.pres)
    h2 = sys["h"].clone()
    u2 = ctx.zeros(d, N)
    ctx.correct(sys, p2, p1, ubd, u2)
    torch.cuda.synchronize()
    _close("A", sys["A"], rec.A)
    _close("u*", us, rec.u_star)
    _close("h*", h1, rec.h1)
    assert rel_p(host(p1), rec.p1) <= TOL
    _close("u**", u1, rec.u1)
    _close("h**", h2, rec.h2)
    assert rel_p(host(p2), rec.p2) <= TOL
    _close("u^{n+1}", u2, rec.u2)

    # ---- oracle adjoint pieces, step by step (the order of step_vjp)
    G = _Grads(geo, np.float64)
    A = rec.A
    hbar2, pb2 = correct_vjp(geo, G, A, rec.p2, w)
    ptot2 = pbar + pb2
    lam2 = pressure_solve_vjp(geo, G, rec, A, rec.p2, ptot2, "direct", 1e-13)
    u1bar, plag2bar = h_rhs_vjp(geo, G, rec, A, rec.h2, rec.u1, rec.p1, hbar2, lam2)
    snap2 = (G.A.copy(), G.b_u.copy(), _oracle_dC(geo, G), G.u_b.copy())
    hbar1, pb1 = correct_vjp(geo, G, A, rec.p1, u1bar)
    ptot1 = plag2bar + pb1
    lam1 = pressure_solve_vjp(geo, G, rec, A, rec.p1, ptot1, "direct", 1e-13)
    usbar, plag1bar = h_rhs_vjp(geo, G, rec, A, rec.h1, rec.u_star, rec.p_n, hbar1, lam1)
    ref = step_vjp(geo, rec, w, pbar)

    # ---- GPU twins in reverse order
    g = ctx.new_system_grad()
    dub = ctx.zeros(d, ctx.NB) if ctx.NB else None
    # corrector 2: u^{n+1} = h** - A^-1 grad p**
    sys["h"].copy_(h2)
    dh2 = ctx.zeros(d, N)
    dp2 = pbd.clone()
    ctx.correct_backward(sys, p2, wd, dh2, dp2, g["dA"])
    torch.cuda.synchronize()
    _close("c2 dh", dh2, hbar2)
    _close("c2 dp", dp2, ptot2)
    du1 = ctx.zeros(d, N)
    dp1 = ctx.zeros(N)
    inf = ctx.solve_pressure_backward(sys, u1, p1, p2, dh2, dp2, du1, dp1, dub, g, o.pres)
    torch.cuda.synchronize()
    assert inf["status"] == 0, inf
    _close("c2 du_in", du1, u1bar)
    _close("c2 dp_lag", dp1, plag2bar, tol=TOL if geo.non_orthogonal else 0.0)
    _close("c2 dA", g["dA"], snap2[0])
    _close("c2 db_u", g["db_u"], snap2[1])
    _close("c2 dC", g["dC"], snap2[2])
    if dub is not None:
        _close("c2 du_b", dub, snap2[3])
    # corrector 1: u** = h* - A^-1 grad p*
    sys["h"].copy_(h1)
    dh1 = ctx.zeros(d, N)
    ctx.correct_backward(sys, p1, du1, dh1, dp1, g["dA"])
    torch.cuda.synchronize()
    _close("c1 dp", dp1, ptot1)
    dus = ctx.zeros(d, N)
    dpn = ctx.zeros(N)
    inf = ctx.solve_pressure_backward(sys, us, pd, p1, dh1, dp1, dus, dpn, dub, g, o.pres)
    torch.cuda.synchronize()
    assert inf["status"] == 0, inf
    _close("c1 du_in", dus, usbar)
    _close("c1 dp_lag", dpn, plag1bar, tol=TOL if geo.non_orthogonal else 0.0)
    # velocity solve and assembly
    inf = ctx.solve_velocity_backward(sys, us, dus, g, o.vel)
    assert inf["status"] == 0, inf
    du_n, dS, dnu = ctx.zeros(d, N), ctx.zeros(d, N), ctx.zeros(N)
    ctx.assemble_backward(ud, nud, ubd, dt, g, du_n, dpn, dS, dnu, dub)
    torch.cuda.synchronize()
    _close("dA", g["dA"], ref["A"])
    _close("du_n", du_n, ref["u_n"])
    _close("dp_n", dpn, ref["p_n"])
    _close("dS", dS, ref["S"])
    _close("dnu", dnu, ref["nu"])
    if dub is not None:
        _close("du_b", dub, ref["u_b"])

    # ---- the same against the whole-step adjoint call
    tape = ctx.new_tape()
    ctx.step(ud, pd, nud, Sd, ubd, dt, o, tape=tape)
    whole = ctx.step_backward(tape, ud, pd, nud, ubd, dt, wd, pbd, o)
    torch.cuda.synchronize()
    for k, v in (("u", du_n), ("p", dpn), ("S", dS), ("nu", dnu)):
        e = rel(host(v), host(whole[k]))
        say("  twins vs piso_step_backward %-2s rel %.2e" % (k, e))
        assert e <= 1e-10, k
