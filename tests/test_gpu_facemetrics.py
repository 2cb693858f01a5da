"""Metrics on the Dirichlet faces (piso_domain_desc.Tb / Jb, App. A.4) on the GPU.

* face metrics equal to the boundary cells' change nothing, bit for bit (forward and
  adjoint), on the vectorised single-block channel and the non-orthogonal 5-block grid;
* with face metrics unlike the cells' (scaled, with cross terms), the step and its
  adjoint against the FP64 oracle (also on the orthogonal channel, where the faces'
  cross terms alone switch the non-orthogonal boundary terms on);
* the outflow update and its adjoint against the oracle;
* argument errors.
"""
import dataclasses

import numpy as np
import pytest
import torch

import cases
from oracle import outflow as oout
from oracle.adjoint import step_vjp
from oracle.piso import Geometry, step as oracle_step
from tests.gpu_common import dev, host, max_elem, rel, rel_p, say, small_cases, tight_opts, random_state
from tests.test_oracle_facemetrics import _with_face_metrics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api as A
    return A


def _run(api, case, prec, seed, backward=True):
    ctx = api.Context(case.domain, prec)
    u, p, S, ub, nu = random_state(case, seed)
    t = ctx.dtype
    if prec == "f64":
        o = tight_opts(ctx)
    else:   # inputs rounded to FP32 once (the oracle upcasts the same values), default solves
        u, p, S, ub, nu = [np.asarray(x, dtype=np.float32).astype(np.float64) for x in (u, p, S, ub, nu)]
        o = ctx.default_opts()
        if prec == "f32":
            o.pres.rtol = 1e-6
    tape = ctx.new_tape()
    u1, p1, _ = ctx.step(dev(u, t), dev(p, t), dev(nu, t), dev(S, t), dev(ub, t), case.dt, o, tape=tape, info=True)
    out = {"u": host(u1), "p": host(p1)}
    if backward:
        rng = np.random.default_rng(seed + 1)
        wu, wp = rng.standard_normal(u.shape), rng.standard_normal(p.shape)
        ctx.adjoint_reset()
        g = ctx.step_backward(tape, dev(u, t), dev(p, t), dev(nu, t), dev(ub, t), case.dt, dev(wu, t), dev(wp, t), o)
        out.update({"g" + k: host(v) for k, v in g.items()})
        out["w"] = (wu, wp)
    return ctx, (u, p, S, ub, nu), out


@pytest.mark.parametrize("name", ["channel_q", "cylinder_q"])
def test_cell_values_on_faces_change_nothing(api, name):
    say("test_cell_values_on_faces_change_nothing", name)
    case = small_cases()[name]
    geo = Geometry(case.domain)
    same = _with_face_metrics(case, 0, Tb=geo.T[:, :, geo.bP].copy(), Jb=geo.J[geo.bP].copy())
    _, _, a = _run(api, case, "f64", 3)
    _, _, b = _run(api, same, "f64", 3)
    for k in a:
        if k != "w":
            assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("name", ["channel_q", "cylinder_q", "sheared"])
def test_step_and_adjoint_vs_oracle(api, name):
    say("test_step_and_adjoint_vs_oracle", name)
    case = _with_face_metrics(small_cases()[name], 5)
    ctx, (u, p, S, ub, nu), out = _run(api, case, "f64", 7)
    assert ctx.non_orthogonal
    geo = Geometry(case.domain)
    rec = oracle_step(geo, u, p, nu, S, case.dt, ub)
    say("  rel u %.2e p %.2e" % (rel(out["u"], rec.u2), rel_p(out["p"], rec.p2)))
    assert rel(out["u"], rec.u2) < 1e-9 and max_elem(out["u"], rec.u2) < 1e-8
    assert rel_p(out["p"], rec.p2) < 1e-9
    wu, wp = out["w"]
    g = step_vjp(geo, rec, wu, wp)
    for k in ("u", "p", "S", "u_b"):
        e = rel(out["g" + k], g[k if k not in ("u", "p") else k + "_n"])
        say("  grad %s %.2e" % (k, e))
        assert e < 1e-8, k
    assert rel(out["gnu"], g["nu"]) < 1e-8


@pytest.mark.parametrize("prec", ["f32", "mixed"])
def test_single_precision_vs_oracle(api, prec):
    say("test_single_precision_vs_oracle", prec)
    case = _with_face_metrics(small_cases()["cylinder_q"], 8)
    _, (u, p, S, ub, nu), out = _run(api, case, prec, 9, backward=False)
    rec = oracle_step(Geometry(case.domain), u, p, nu, S, case.dt, ub)
    say("  rel u %.2e p %.2e" % (rel(out["u"], rec.u2), rel_p(out["p"], rec.p2)))
    assert rel(out["u"], rec.u2) < (1e-5 if prec == "f32" else 1e-8)
    assert rel_p(out["p"], rec.p2) < (1e-4 if prec == "f32" else 1e-7)


def test_outflow_vs_oracle(api):
    say("test_outflow_vs_oracle")
    case = _with_face_metrics(cases.open_channel(24, 12), 11, cross=0.0)
    geo = Geometry(case.domain)
    ctx = api.Context(case.domain, "f64")
    t = ctx.dtype
    rng = np.random.default_rng(12)
    u = case.u0 + 0.1 * rng.standard_normal(case.u0.shape)
    ub = case.u_b + 0.05 * rng.standard_normal(case.u_b.shape)
    gbar = rng.standard_normal(ub.shape)
    mask, u_m = case.extra["outflow"], case.extra["u_m"]
    m = ctx.outflow_mask(mask)
    out = ctx.outflow_update(dev(u, t), dev(ub, t), m, u_m, case.dt)
    dub, du = ctx.outflow_update_backward(dev(u, t), dev(ub, t), m, u_m, case.dt, dev(gbar, t))
    ref = oout.update(geo, u, ub, mask, u_m, case.dt)
    du_o, dub_o = oout.update_vjp(geo, u, ub, mask, u_m, case.dt, gbar)
    assert rel(host(out), ref) < 1e-13
    assert rel(host(dub), dub_o) < 1e-12 and rel(host(du), du_o) < 1e-12


def test_face_metric_errors(api):
    say("test_face_metric_errors")
    case = small_cases()["channel_q"]
    geo = Geometry(case.domain)
    bad = _with_face_metrics(case, 1, Tb=geo.T[:, :, geo.bP].copy(), Jb=-geo.J[geo.bP])
    with pytest.raises(RuntimeError, match="Jb"):
        api.Context(bad.domain, "f64")
    short = dataclasses.replace(case.domain, Tb=geo.T[:, :, geo.bP][:, :, :-1].copy(), Jb=geo.J[geo.bP][:-1].copy())
    with pytest.raises(ValueError, match="face metrics"):
        api.Context(short, "f64")
