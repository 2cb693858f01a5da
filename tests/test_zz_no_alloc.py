"""The allocation-free velocity solve (piso_solve_velocity_noalloc) against
piso_solve_velocity: same kernels on the same inputs, so the same bits, on consecutive
calls of decreasing size that share the fixed per-GPU workspace; sizes beyond the
workspace and MIXED contexts are refused before any launch."""
import numpy as np
import pytest
import torch

import cases
from tests.gpu_common import dev, random_state, say

pytestmark = pytest.mark.gpu


def _one(api, case, prec, seed):
    ctx = api.Context(case.domain, prec)
    t = ctx.dtype
    u, p, S, ub, nu = random_state(case, seed)
    ud = dev(u, t)
    sys = ctx.new_system()
    ctx.assemble(sys, ud, dev(p, t), dev(nu, t), dev(S, t), dev(ub, t), case.dt)
    o = ctx.default_opts().vel
    o.rtol = 1e-10 if prec == "f64" else 1e-6
    x_ref = ud.clone()
    i_ref = ctx.solve_velocity(sys, x_ref, o)
    x = ud.clone()
    i_new = ctx.solve_velocity_noalloc(sys, x, o)
    torch.cuda.synchronize()
    say("  %s N=%d %s: iters %d / %d, residual %.3e / %.3e" % (case.name, ctx.N, prec, i_ref["iters"],
                                                              i_new["iters"], i_ref["rel_residual"],
                                                              i_new["rel_residual"]))
    assert i_ref["status"] == 0
    assert i_new == i_ref
    assert torch.equal(x, x_ref)


def test_noalloc_velocity_matches_context_solve():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api
    say("test_noalloc_velocity_matches_context_solve")
    # two calls in a row per precision, the second on a smaller grid
    for prec in ("f64", "f32"):
        _one(api, cases.channel(64, 48, 40), prec, 1)
        _one(api, cases.cylinder_oh(16, 8, 4), prec, 2)


def test_noalloc_velocity_refuses_beyond_workspace():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api
    for prec, case in (("f64", cases.channel(96, 96, 96)), ("mixed", cases.channel(12, 10, 8))):
        ctx = api.Context(case.domain, prec)
        sys = ctx.new_system()
        x = ctx.zeros(ctx.dim, ctx.N)
        with pytest.raises(api.PisoError) as e:
            ctx.solve_velocity_noalloc(sys, x, ctx.default_opts().vel)
        assert e.value.code == -1
        say("  refused %s N=%d: %s" % (prec, ctx.N, e.value))
