"""Online plane statistics on the GPU against the oracle (Sec. 2.5)."""
import numpy as np
import pytest
import torch

import cases
from oracle import stats as ostats
from tests.gpu_common import dev, host, rel, say

pytestmark = pytest.mark.gpu


def _api():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api
    return api


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_accumulate_finalize_backward_vs_oracle(prec, axis):
    api = _api()
    case = cases.channel(12, 10, 8)
    dims = case.domain.blocks[0]
    ctx = api.Context(case.domain, prec)
    t = ctx.dtype
    rng = np.random.default_rng(30 + axis)
    us = [case.u0 + 0.3 * rng.standard_normal(case.u0.shape) for _ in range(4)]
    if prec == "f32":
        us = [u.astype(np.float32).astype(np.float64) for u in us]
    st = ostats.empty_state(dims[axis], 3)
    for u in us:
        st = ostats.accumulate(st, u, dims, axis)
    m_ref, c_ref = ostats.finalize(st)
    mbar = rng.standard_normal(m_ref.shape)
    cbar = rng.standard_normal(c_ref.shape)
    g_ref = [ostats.stats_vjp(st, u, dims, axis, mbar, cbar) for u in us]
    ud = [dev(u, t) for u in us]
    state = ctx.stats_state(axis)
    for u in ud:
        ctx.stats_accumulate(u, state, axis)
    mean, cov = ctx.stats_finalize(state, axis)
    em, ec = rel(host(mean), m_ref), rel(host(cov), c_ref)
    gs = [ctx.stats_backward(u, state, dev(mbar, torch.float64), dev(cbar, torch.float64), axis) for u in ud]
    eg = max(rel(host(g), r) for g, r in zip(gs, g_ref))
    say("%s axis %d: mean %.2e cov %.2e grad %.2e" % (prec, axis, em, ec, eg))
    assert em < 1e-13 and ec < 1e-12
    assert eg < (1e-13 if prec == "f64" else 1e-6)


def test_autograd_statistics_loss_through_rollout():
    """Gradient of a statistics loss over a 3-step F64 rollout with respect to the
    source, against central differences."""
    api = _api()
    case = cases.channel(12, 10, 8)
    ctx = api.Context(case.domain, "f64")
    t = ctx.dtype
    o = ctx.default_opts()
    o.vel.rtol = o.pres.rtol = 1e-13
    u0, p0, nu, ub = dev(case.u0, t), dev(case.p0, t), dev([case.nu], t), dev(case.u_b, t)
    rng = np.random.default_rng(31)
    S0 = dev(case.S, t)
    u_hat = dev(rng.standard_normal(10), torch.float64)

    def loss_of(S, grad):
        traj = api.rollout(ctx, u0, p0, S, nu, ub, case.dt, 3, opts=o, return_all=True)
        mean, cov = api.plane_statistics(ctx, [u for u, _ in traj], axis=1)
        return ((mean[:, 0] - u_hat) ** 2).mean() + ((cov[:, 1] - 0.01) ** 2).mean()

    S = S0.clone().requires_grad_(True)
    L = loss_of(S, True)
    (gS,) = torch.autograd.grad(L, [S])
    cells = [(0, 17), (0, 455), (1, 300), (2, 901)]
    for comp, cell in cells:
        eps = 1e-5
        Sp, Sm = S0.clone(), S0.clone()
        Sp[comp, cell] += eps
        Sm[comp, cell] -= eps
        with torch.no_grad():
            fd = (float(loss_of(Sp, False)) - float(loss_of(Sm, False))) / (2 * eps)
        an = float(gS[comp, cell])
        say("FD (%d, %d): fd %.8e adjoint %.8e" % (comp, cell, fd, an))
        # central differences of a loss converged to rtol 1e-13 carry an absolute noise
        # of about 1e-13 |L| / eps = 1e-8 here
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-8


def test_rejects_multiblock():
    api = _api()
    ctx = api.Context(cases.cylinder_oh(16, 6, 5).domain, "f64")
    with pytest.raises(api.PisoError):
        ctx.stats_size(1)
