"""Advective outflow boundary on the GPU against the oracle (forward, adjoint, and
rollouts that update the boundary before every step)."""
import numpy as np
import pytest
import torch

import cases
from oracle import outflow as oout
from oracle.adjoint import step_vjp
from oracle.piso import Geometry, step as oracle_step
from tests.gpu_common import dev, host, rel, say, tight_opts

pytestmark = pytest.mark.gpu


def _api():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api
    return api


def _cases():
    op = cases.open_channel(24, 12)
    cyl = cases.cylinder_oh(16, 6, 5)
    cyl.extra["outflow"] = cases.segment_mask(cyl.domain, lambda si: cyl.domain.sides[si].block == 1)
    cyl.extra["u_m"] = np.array([1.0, 0.0])
    return {"open_channel": op, "cylinder": cyl}


@pytest.mark.parametrize("name", ["open_channel", "cylinder"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_update_and_adjoint_vs_oracle(name, prec):
    api = _api()
    case = _cases()[name]
    geo = Geometry(case.domain)
    rng = np.random.default_rng(21)
    u = case.u0 + 0.3 * rng.standard_normal(case.u0.shape)
    ub = case.u_b + 0.2 * rng.standard_normal(case.u_b.shape)
    gbar = rng.standard_normal(ub.shape)
    mask, u_m, dt = case.extra["outflow"], case.extra["u_m"], case.dt
    ref = oout.update(geo, u, ub, mask, u_m, dt)
    rdu, rdub = oout.update_vjp(geo, u, ub, mask, u_m, dt, gbar)
    ctx = api.Context(case.domain, prec)
    t = ctx.dtype
    m = ctx.outflow_mask(mask)
    out = ctx.outflow_update(dev(u, t), dev(ub, t), m, u_m, dt)
    dub, du = ctx.outflow_update_backward(dev(u, t), dev(ub, t), m, u_m, dt, dev(gbar, t))
    e0, e1, e2 = rel(host(out), ref), rel(host(dub), rdub), rel(host(du), rdu)
    say("%s %s: update %.2e, du_b %.2e, du %.2e" % (name, prec, e0, e1, e2))
    tol = 1e-13 if prec == "f64" else 2e-6
    assert e0 < tol and e1 < tol and e2 < tol
    # zero net boundary flux of the result
    _, w = oout.face_coefficients(geo, u_m, dt)
    assert abs(np.sum(w * host(out))) < (1e-12 if prec == "f64" else 1e-5) * np.sum(np.abs(w * host(out)))


def test_outflow_accumulates_du_and_in_place():
    api = _api()
    case = _cases()["open_channel"]
    ctx = api.Context(case.domain, "f64")
    t = ctx.dtype
    m = ctx.outflow_mask(case.extra["outflow"])
    u, ub = dev(case.u0, t), dev(case.u_b, t)
    g = torch.randn_like(ub)
    base = torch.randn_like(u)
    _, du0 = ctx.outflow_update_backward(u, ub, m, case.extra["u_m"], case.dt, g)
    dub, du1 = ctx.outflow_update_backward(u, ub, m, case.extra["u_m"], case.dt, g, du=base.clone())
    assert torch.allclose(du1, base + du0, rtol=0, atol=1e-15)
    ref = ctx.outflow_update(u, ub, m, case.extra["u_m"], case.dt)
    ub2 = ub.clone()
    ctx.outflow_update(u, ub2, m, case.extra["u_m"], case.dt, out=ub2)
    assert torch.equal(ub2, ref)


def test_rollout_with_outflow_vs_oracle_chain():
    """Six F64 steps of the open channel with the outflow update before each step,
    against the oracle's chain; then the gradient of <w, u^6> with respect to the
    initial boundary values and the source against the oracle's adjoint chain, with and
    without step checkpointing."""
    api = _api()
    case = _cases()["open_channel"]
    geo = Geometry(case.domain)
    mask, u_m, dt = case.extra["outflow"], case.extra["u_m"], case.dt
    rng = np.random.default_rng(22)
    u0 = case.u0 + 0.05 * rng.standard_normal(case.u0.shape)
    S = 0.1 * rng.standard_normal(case.u0.shape)
    w = rng.standard_normal(case.u0.shape)
    n = 6
    # oracle chain with records
    recs, ubs = [], [case.u_b]
    u, p, ub = u0, case.p0, case.u_b
    for _ in range(n):
        ubn = oout.update(geo, u, ub, mask, u_m, dt)
        rec = oracle_step(geo, u, p, case.nu, S, dt, ubn)
        recs.append((u, ub, ubn, rec))
        u, p, ub = rec.u2, rec.p2, ubn
    uT_ref = u
    # oracle adjoint chain
    gu, gp, gb = w, np.zeros(geo.N), np.zeros_like(case.u_b)
    dS_ref = np.zeros_like(S)
    for q in range(n - 1, -1, -1):
        un, ubprev, ubused, rec = recs[q]
        g = step_vjp(geo, rec, gu, gp, mode="direct", rtol=1e-13)
        dS_ref += g["S"]
        du_o, gb = oout.update_vjp(geo, un, ubprev, mask, u_m, dt, g["u_b"] + gb)
        gu, gp = g["u_n"] + du_o, g["p_n"]
    ctx = api.Context(case.domain, "f64")
    t = ctx.dtype
    o = tight_opts(ctx)
    m = ctx.outflow_mask(mask)
    for k in (0, 2):
        ub_t = dev(case.u_b, t).requires_grad_(True)
        S_t = dev(S, t).requires_grad_(True)
        uT, pT, ubT = api.rollout(ctx, dev(u0, t), dev(case.p0, t), S_t, dev([case.nu], t), ub_t, dt, n,
                                  checkpoint_every=k, opts=o, outflow=(m, u_m))
        e_u = rel(host(uT), uT_ref)
        e_b = rel(host(ubT), ub)
        gub, gS = torch.autograd.grad((uT * dev(w, t)).sum(), [ub_t, S_t])
        e_gb, e_gS = rel(host(gub), gb), rel(host(gS), dS_ref)
        say("checkpoint %d: u %.2e u_b %.2e | grad u_b %.2e grad S %.2e" % (k, e_u, e_b, e_gb, e_gS))
        assert e_u < 1e-9 and e_b < 1e-9
        assert e_gb < 1e-7 and e_gS < 1e-7
