"""GPU rollouts: autograd Function, step checkpointing, gradient paths, determinism,
quad-vs-generic kernels, and finite differences through a multi-block rollout."""
import os

import numpy as np
import pytest
import torch

import cases
from oracle.adjoint import step_vjp
from oracle.piso import Geometry, step as oracle_step
from tests.gpu_common import dev, host, rel, rel_p, say, small_cases, tight_opts, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api as A
    return A


def _inputs(ctx, case, seed, scale=0.1):
    u, p, S, ub, nu = random_state(case, seed, scale)
    t = ctx.dtype
    return (u, p, S, ub, nu), [dev(x, t) for x in (u, p, S, ub)] + [dev(np.array([case.nu]), t)]


@pytest.mark.parametrize("name", ["channel_q", "cylinder_q"])
def test_quad_matches_generic(api, name):
    say("test_quad_matches_generic", name)
    case = small_cases()[name]
    outs = []
    for env in ("0", "1"):
        os.environ["PISO_NO_QUAD"] = env
        try:
            ctx = api.Context(case.domain, "f64")
        finally:
            os.environ.pop("PISO_NO_QUAD", None)
        _, (u, p, S, ub, nu) = _inputs(ctx, case, 3)
        o = tight_opts(ctx)
        u1, p1, info = ctx.step(u, p, nu, S, ub, case.dt, o, info=True)
        outs.append((host(u1), host(p1), [q["iters"] for q in info["pres"]]))
    assert rel(outs[0][0], outs[1][0]) < 1e-11
    assert rel_p(outs[0][1], outs[1][1]) < 1e-10
    # the multigrid preconditioner (vectorised and generic update/restriction kernels)
    # is the same linear map up to rounding: the same CG iteration counts
    say("pressure CG iterations quad %s generic %s" % (outs[0][2], outs[1][2]))
    assert all(abs(a - b) <= 1 for a, b in zip(outs[0][2], outs[1][2]))


def test_deterministic(api):
    say("test_deterministic")
    case = cases.channel(16, 12, 8)
    ctx = api.Context(case.domain, "f32")
    _, (u, p, S, ub, nu) = _inputs(ctx, case, 4)
    a = ctx.step(u, p, nu, S, ub, case.dt)
    b = ctx.step(u, p, nu, S, ub, case.dt)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("name", ["channel_q", "cylinder_q"])
def test_rollout_matches_oracle_chain(api, name):
    """3-step rollout through the autograd Function vs the chained oracle adjoint."""
    say("test_rollout_matches_oracle_chain", name)
    case = small_cases()[name]
    ctx = api.Context(case.domain, "f64")
    (u0, p0, S0, ub0, _), (u, p, S, ub, nu) = _inputs(ctx, case, 5)
    o = tight_opts(ctx)
    rng = np.random.default_rng(6)
    w = rng.standard_normal(u0.shape)
    S_ = S.clone().requires_grad_(True)
    u_ = u.clone().requires_grad_(True)
    nu_ = nu.clone().requires_grad_(True)
    uT, pT = api.rollout(ctx, u_, p, S_, nu_, ub, case.dt, 3, checkpoint_every=0, opts=o)
    L = (uT * dev(w, ctx.dtype)).sum()
    gS, gu, gnu = torch.autograd.grad(L, [S_, u_, nu_])
    geo = Geometry(case.domain)
    recs, uu, pp = [], u0, p0
    for _ in range(3):
        r = oracle_step(geo, uu, pp, case.nu, S0, case.dt, ub0)
        recs.append(r)
        uu, pp = r.u2, r.p2
    gu_o, gp_o = w, np.zeros(geo.N)
    dS, dnu = 0.0, 0.0
    for r in reversed(recs):
        g = step_vjp(geo, r, gu_o, gp_o)
        gu_o, gp_o = g["u_n"], g["p_n"]
        dS = dS + g["S"]
        dnu = dnu + g["nu"].sum()
    assert rel(host(gS), dS) < 1e-8
    assert rel(host(gu), gu_o) < 1e-8
    assert abs(float(host(gnu)[0]) - dnu) <= 1e-8 * abs(dnu)


def test_checkpointing_is_exact(api):
    """Recomputing segment tapes reproduces the stored-tape adjoint chain bit for bit
    (the initial-state gradient); gradients of parameters shared by all steps (S) are
    sums whose order differs between segmentings, so they agree to rounding."""
    say("test_checkpointing_is_exact")
    case = small_cases()["cylinder_q"]
    ctx = api.Context(case.domain, "f32")
    _, (u, p, S, ub, nu) = _inputs(ctx, case, 7)
    w = torch.randn_like(u)
    grads = []
    for k in (0, 2, 3):
        S_ = S.clone().requires_grad_(True)
        u_ = u.clone().requires_grad_(True)
        uT, _ = api.rollout(ctx, u_, p, S_, nu, ub, case.dt, 6, checkpoint_every=k)
        grads.append(torch.autograd.grad((uT * w).sum(), [u_, S_]))
    for g in grads[1:]:
        assert torch.equal(grads[0][0], g[0])
        assert rel(host(g[1]), host(grads[0][1])) < 1e-6


def test_fd_through_multiblock_rollout(api):
    """Central differences of a 6-step rollout loss on the non-orthogonal 5-block grid
    (FP64, checkpoint every 2) against the adjoint gradient with respect to S."""
    say("test_fd_through_multiblock_rollout")
    case = small_cases()["cylinder_q"]
    ctx = api.Context(case.domain, "f64")
    _, (u, p, S, ub, nu) = _inputs(ctx, case, 8)
    o = tight_opts(ctx, 1e-14, 1e-14)
    w = dev(np.random.default_rng(9).standard_normal((2, ctx.N)), torch.float64)
    S_ = S.clone().requires_grad_(True)
    uT, _ = api.rollout(ctx, u, p, S_, nu, ub, case.dt, 6, checkpoint_every=2, opts=o)
    (gS,) = torch.autograd.grad((uT * w).sum(), [S_])

    def loss(Sx):
        with torch.no_grad():
            uu, pp = u, p
            for _ in range(6):
                uu, pp = ctx.step(uu, pp, nu, Sx, ub, case.dt, o)
            return float((uu * w).sum())

    rng = np.random.default_rng(10)
    for _ in range(6):
        comp, cell = int(rng.integers(2)), int(rng.integers(ctx.N))
        eps = 1e-4
        Sp, Sm = S.clone(), S.clone()
        Sp[comp, cell] += eps
        Sm[comp, cell] -= eps
        fd = (loss(Sp) - loss(Sm)) / (2 * eps)
        an = float(gS[comp, cell])
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-2), (comp, cell, fd, an)


def test_gradient_path_flags(api):
    """Skipping the adjoint solves (Sec. 2.4) matches the oracle's bypass gradients."""
    say("test_gradient_path_flags")
    case = small_cases()["channel_q"]
    ctx = api.Context(case.domain, "f64")
    (u0, p0, S0, ub0, nu0), (u, p, S, ub, nu) = _inputs(ctx, case, 11)
    o = tight_opts(ctx)
    geo = Geometry(case.domain)
    rec = oracle_step(geo, u0, p0, case.nu, S0, case.dt, ub0)
    w = np.random.default_rng(12).standard_normal(u0.shape)
    for flags, kw in ((1, dict(skip_velocity_solve=True)), (2, dict(skip_pressure_solve=True)),
                      (3, dict(skip_velocity_solve=True, skip_pressure_solve=True))):
        o.grad_path_flags = flags
        tape = ctx.new_tape()
        ctx.step(u, p, nu, S, ub, case.dt, o, tape=tape)
        g = ctx.step_backward(tape, u, p, nu, ub, case.dt, dev(w, torch.float64), None, o)
        gr = step_vjp(geo, rec, w, np.zeros(geo.N), **kw)
        assert rel(host(g["S"]), gr["S"]) < 1e-8, flags
        assert rel(host(g["u"]), gr["u_n"]) < 1e-8, flags


def test_adjoint_warm_start(api):
    """The adjoint pressure solves of step_backward start from the previous call's
    solutions (adjoint_warm_start, the default): a repeated call converges at once and
    agrees to solver tolerance; adjoint_reset restores the cold-start result bit for bit;
    with the option off every call is cold."""
    say("test_adjoint_warm_start")
    case = small_cases()["channel_q"]
    ctx = api.Context(case.domain, "f64")
    _, (u, p, S, ub, nu) = _inputs(ctx, case, 8)
    o = tight_opts(ctx)
    assert o.adjoint_warm_start == 1
    tape = ctx.new_tape()
    ctx.step(u, p, nu, S, ub, case.dt, o, tape=tape)
    rng = np.random.default_rng(9)
    du1 = dev(rng.standard_normal(u.shape), ctx.dtype)
    dp1 = dev(rng.standard_normal(p.shape), ctx.dtype)

    def bwd():
        g, inf = ctx.step_backward(tape, u, p, nu, ub, case.dt, du1, dp1, o, info=True)
        return {k: host(v) for k, v in g.items() if v is not None}, [q["iters"] for q in inf["pres"]]

    ctx.adjoint_reset()
    g1, it1 = bwd()
    g2, it2 = bwd()
    say("adjoint pressure iterations cold %s, warm repeat %s" % (it1, it2))
    assert all(b < a for a, b in zip(it1, it2))
    for k in g1:
        assert rel(g2[k], g1[k]) < 1e-9
    ctx.adjoint_reset()
    g3, it3 = bwd()
    assert it3 == it1
    for k in g1:
        assert np.array_equal(g3[k], g1[k])
    o.adjoint_warm_start = 0
    g4, it4 = bwd()
    g5, it5 = bwd()
    assert it4 == it1 and it5 == it1
    for k in g1:
        assert np.array_equal(g4[k], g1[k]) and np.array_equal(g5[k], g1[k])


def test_adjoint_history_isolated_between_rollouts(api):
    """The adjoint warm start never crosses from one backward pass to another: a
    rollout's gradient is bit for bit the same whatever was differentiated before it,
    also when the loss uses an earlier state than the last (then the rollout's final
    step never runs its backward), and a stand-alone step's too."""
    say("test_adjoint_history_isolated_between_rollouts")
    case = small_cases()["channel_q"]
    ctx = api.Context(case.domain, "f64")
    _, (u, p, S, ub, nu) = _inputs(ctx, case, 13)
    w = torch.randn_like(u)

    def grads_mid(k):
        S_ = S.clone().requires_grad_(True)
        traj = api.rollout(ctx, u, p, S_, nu, ub, case.dt, 3, checkpoint_every=k, return_all=True)
        (g,) = torch.autograd.grad((traj[0][0] * w).sum() + (traj[1][0] * w).sum(), [S_])
        return g

    def grads_other():
        S_ = (2.0 * S).requires_grad_(True)
        uT, _ = api.rollout(ctx, u, p, S_, nu, ub, case.dt, 3)
        torch.autograd.grad((uT * uT).sum(), [S_])

    def grads_step():
        S_ = S.clone().requires_grad_(True)
        u1, _ = api.step(ctx, u, p, S_, nu, ub, case.dt)
        return torch.autograd.grad((u1 * w).sum(), [S_])[0]

    for k in (0, 1):
        a = grads_mid(k)
        grads_other()
        b = grads_mid(k)
        assert torch.equal(a, b), k
    a = grads_step()
    grads_other()
    b = grads_step()
    assert torch.equal(a, b)


def test_rollout_warmup(api):
    """warmup steps run without a tape before the differentiated ones: the same final
    state as running them by hand, and the gradient of the rollout that starts there.
    Without the pressure extrapolation a rollout after warm-up equals a rollout started
    from the warmed-up state; with it, the chain of previous pressures runs on through
    the warm-up, so the states equal those of stand-alone steps chained by hand."""
    say("test_rollout_warmup")
    case = small_cases()["cylinder_q"]
    ctx = api.Context(case.domain, "f64")
    _, (u, p, S, ub, nu) = _inputs(ctx, case, 14)
    o = tight_opts(ctx)
    w = torch.randn_like(u)
    S1 = S.clone().requires_grad_(True)
    uT, pT = api.rollout(ctx, u, p, S1, nu, ub, case.dt, 2, warmup=3, opts=o, extrapolate=False)
    (g1,) = torch.autograd.grad((uT * w).sum(), [S1])
    uu, pp = u, p
    for _ in range(3):
        uu, pp = ctx.step(uu, pp, nu, S, ub, case.dt, o)
    S2 = S.clone().requires_grad_(True)
    uT2, pT2 = api.rollout(ctx, uu, pp, S2, nu, ub, case.dt, 2, opts=o, extrapolate=False)
    (g2,) = torch.autograd.grad((uT2 * w).sum(), [S2])
    assert torch.equal(uT.detach(), uT2.detach()) and torch.equal(pT.detach(), pT2.detach())
    assert torch.equal(g1, g2)
    uE, pE = api.rollout(ctx, u, p, S, nu, ub, case.dt, 2, warmup=3, opts=o)
    uu, pp, uv, pv, pvs = u, p, None, None, None
    for _ in range(5):
        pst = torch.empty_like(pp)
        u1, p1 = ctx.step(uu, pp, nu, S, ub, case.dt, o, p_prev=pv, p_prev_star=pvs, p_star_out=pst, u_prev=uv)
        uv, pv, pvs, uu, pp = uu, pp, pst, u1, p1
    assert torch.equal(uE.detach(), uu) and torch.equal(pE.detach(), pp)


@pytest.mark.parametrize("name", ["tgv16", "cavity12", "channel_q", "cylinder_q"])
def test_extrapolated_start_matches_oracle(api, name):
    """A step given earlier fields (u_prev, p_prev, p_prev_star: its linear solves start
    from them) reaches the oracle's step to the solver tolerance, whatever they are: the
    start of a converged Krylov solve does not enter the result.  p_star_out receives the
    first corrector's pressure, which the tape holds too."""
    say("test_extrapolated_start_matches_oracle", name)
    case = small_cases()[name]
    ctx = api.Context(case.domain, "f64")
    (u0, p0, S0, ub0, _), (u, p, S, ub, nu) = _inputs(ctx, case, 21)
    o = tight_opts(ctx)
    ref = oracle_step(Geometry(case.domain), u0, p0, case.nu, S0, case.dt, ub0)
    rng = np.random.default_rng(22)
    t = ctx.dtype
    near = (u0 + 0.05 * rng.standard_normal(u0.shape), p0 + 0.05 * rng.standard_normal(p0.shape),
            p0 + 0.05 * rng.standard_normal(p0.shape))
    far = (rng.standard_normal(u0.shape), rng.standard_normal(p0.shape), rng.standard_normal(p0.shape))
    for uv, pv, pvs in (near, far, (None, near[1], None), (far[0], None, far[2])):
        pst = torch.empty_like(p)
        tape = ctx.new_tape()
        u1, p1, info = ctx.step(u, p, nu, S, ub, case.dt, o, info=True, tape=tape,
                                u_prev=None if uv is None else dev(uv, t),
                                p_prev=None if pv is None else dev(pv, t),
                                p_prev_star=None if pvs is None else dev(pvs, t), p_star_out=pst)
        assert info["vel"]["status"] == 0, info
        assert info["pres"][0]["status"] == 0 and info["pres"][1]["status"] == 0, info
        assert rel(host(u1), ref.u2) < 1e-9
        assert rel_p(host(p1), ref.p2) < 1e-9
        assert rel_p(host(pst), ref.p1) < 1e-9
        N, d = ctx.N, ctx.dim
        off = 2 * N + 5 * d * N   # A, C, P_f, D^-1, u*, h* precede p* on the tape
        assert torch.equal(pst, tape[off:off + N])
    with pytest.raises(ValueError):
        ctx.step(u, p, nu, S, ub, case.dt, o, p_prev=p[:-1])
    with pytest.raises(RuntimeError, match="p_star_out"):
        ctx.step(u, p, nu, S, ub, case.dt, o, p_prev=p.clone(), p_star_out=p)


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_extrapolated_start_saves_iterations(api, prec):
    """On a developed flow, starts from the previous step's fields save pressure
    iterations in both correctors and velocity iterations; the rollout's result agrees
    with the unextrapolated one to the solver tolerance, and a rollout of stand-alone
    steps with the chained starts equals api.rollout's chain bit for bit, checkpointed
    or not."""
    say("test_extrapolated_start_saves_iterations", prec)
    case = cases.channel(32, 24, 16)
    ctx = api.Context(case.domain, prec)
    t = ctx.dtype
    u, p, S, ub = (dev(x, t) for x in (case.u0, case.p0, case.S, case.u_b))
    nu = dev(np.array([case.nu]), t)
    o = ctx.default_opts()
    with torch.no_grad():
        for _ in range(10):                 # let the pressure develop from p0 = 0
            u, p = ctx.step(u, p, nu, S, ub, case.dt, o)
        runs = {}
        for extra in (False, True):
            uu, pp, uv, pv, pvs, its = u, p, None, None, None, []
            for _ in range(8):
                pst = torch.empty_like(pp)
                u1, p1, inf = ctx.step(uu, pp, nu, S, ub, case.dt, o, info=True, p_star_out=pst,
                                       p_prev=pv if extra else None, p_prev_star=pvs if extra else None,
                                       u_prev=uv if extra else None)
                uv, pv, pvs, uu, pp = uu, pp, pst, u1, p1
                its.append([q["iters"] for q in inf["pres"]] + [inf["vel"]["iters"]])
            runs[extra] = (uu, pp, np.array(its))
        say("CG iterations per corrector, plain %s extrapolated %s" % (runs[False][2].tolist(), runs[True][2].tolist()))
        plain, extra = runs[False][2][2:].sum(axis=0), runs[True][2][2:].sum(axis=0)
        assert extra[0] < plain[0] and extra[1] < plain[1] and extra[2] <= plain[2]
        assert rel(host(runs[True][0]), host(runs[False][0])) < 1e-5
        uT, pT = api.rollout(ctx, u, p, S, nu, ub, case.dt, 8, opts=o)
        assert torch.equal(uT, runs[True][0]) and torch.equal(pT, runs[True][1])
        uC, pC = api.rollout(ctx, u, p, S, nu, ub, case.dt, 8, checkpoint_every=3, opts=o)
        assert torch.equal(uC, uT) and torch.equal(pC, pT)
        uN, _ = api.rollout(ctx, u, p, S, nu, ub, case.dt, 8, opts=o, extrapolate=False)
        assert torch.equal(uN, runs[False][0])


@pytest.mark.parametrize("ncorr", [1, 3])
def test_solve_starts_with_other_corrector_counts(api, ncorr):
    """With one or three correctors the starts still only move where the solves begin:
    the result equals the step without them to the solver tolerance, and p_star_out holds
    the first corrector's pressure (with one corrector, the step's output pressure)."""
    say("test_solve_starts_with_other_corrector_counts", ncorr)
    case = small_cases()["cylinder_q"]
    ctx = api.Context(case.domain, "f64")
    _, (u, p, S, ub, nu) = _inputs(ctx, case, 31)
    o = tight_opts(ctx)
    o.n_correctors = ncorr
    g = torch.Generator(device=u.device).manual_seed(32)
    u_prev = u + 0.01 * torch.randn(u.shape, generator=g, device=u.device, dtype=u.dtype)
    p_prev = p + 0.01 * torch.randn(p.shape, generator=g, device=p.device, dtype=p.dtype)
    p_prev_star = p + 0.01 * torch.randn(p.shape, generator=g, device=p.device, dtype=p.dtype)
    u0, p0 = ctx.step(u, p, nu, S, ub, case.dt, o)
    pst = torch.empty_like(p)
    u1, p1 = ctx.step(u, p, nu, S, ub, case.dt, o, u_prev=u_prev, p_prev=p_prev, p_prev_star=p_prev_star,
                      p_star_out=pst)
    assert rel(host(u1), host(u0)) < 1e-10 and rel_p(host(p1), host(p0)) < 1e-9
    if ncorr == 1:
        assert torch.equal(pst, p1)
    else:
        o1 = tight_opts(ctx)
        o1.n_correctors = 1
        _, pstar_ref = ctx.step(u, p, nu, S, ub, case.dt, o1)   # corrector 1 alone
        assert rel_p(host(pst), host(pstar_ref)) < 1e-9
