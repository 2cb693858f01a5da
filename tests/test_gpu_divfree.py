"""Divergence-free gradient modification (eq. SgradPsgrad) on the GPU against the oracle."""
import numpy as np
import pytest
import torch

import cases
from oracle.divfree import divfree_gradient
from oracle.piso import Geometry
from tests.gpu_common import dev, host, rel, rel_p, say, small_cases

pytestmark = pytest.mark.gpu


def _api():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api
    return api


@pytest.mark.parametrize("name", ["channel", "two_block", "cylinder", "sheared", "channel_q"])
@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
def test_divfree_gradient_vs_oracle(name, prec):
    api = _api()
    case = small_cases()[name]
    geo = Geometry(case.domain)
    rng = np.random.default_rng(40)
    S = rng.standard_normal(case.u0.shape)
    gS = rng.standard_normal(case.u0.shape)
    if prec != "f64":
        S = S.astype(np.float32).astype(np.float64)
        gS = gS.astype(np.float32).astype(np.float64)
    g_ref, p_ref = divfree_gradient(geo, S, gS, 0.7)
    ctx = api.Context(case.domain, prec)
    t = ctx.dtype
    o = ctx.default_opts().pres
    if prec == "f64":
        o.rtol = 1e-13
    g, p, info = ctx.divfree_gradient(dev(S, t), dev(gS, t), 0.7, o, info=True)
    eg, ep = rel(host(g) - gS, g_ref - gS), rel_p(host(p), p_ref)
    say("%s %s: lambda grad p rel %.2e, p rel %.2e, iters %d" % (name, prec, eg, ep, info["iters"]))
    assert info["status"] == 0
    tol = {"f64": 1e-10, "mixed": 1e-6, "f32": 1e-5}[prec]
    assert eg < tol and ep < tol


def test_divfree_hook_in_autograd():
    api = _api()
    case = small_cases()["channel_q"]
    ctx = api.Context(case.domain, "f64")
    t = ctx.dtype
    rng = np.random.default_rng(41)
    S = dev(rng.standard_normal(case.u0.shape), t).requires_grad_(True)
    w = dev(rng.standard_normal(case.u0.shape), t)
    Sm = api.divfree_gradient_hook(ctx, S, 0.5)
    assert torch.equal(Sm, S)
    (g,) = torch.autograd.grad((Sm * w).sum(), [S])
    ref, _ = ctx.divfree_gradient(S.detach(), w, 0.5)
    assert torch.allclose(g, ref, rtol=0, atol=0)
    g0, _ = ctx.divfree_gradient(S.detach(), w, 0.0)
    assert torch.equal(g0, w)
