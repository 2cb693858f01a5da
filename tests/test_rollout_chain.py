"""Host logic of api.rollout's chained solve starts (no GPU).

A stand-in context records what every step receives: the previous step's input
velocity and pressure (u_prev, p_prev) and its first-corrector pressure (p_prev_star,
which the step before wrote through p_star_out).  The chain must be the same for single
steps, for checkpointed segments (also when they recompute their steps in the backward),
for warm-up steps and with the outflow update, and absent with extrapolate=False.
"""
import pytest
import torch

from paper_2505_16992_amd import api


class _Recorder:
    """Deterministic CPU stand-in for Context: u1 = u + 1 + S, p1 = 2 p + 1,
    p* = p + 0.5; the backward passes gradients through unchanged."""

    def __init__(self):
        self.calls = []   # (phase, u, p, u_prev, p_prev, p_prev_star) of every step
        self._adj_owner = None
        self.phase = "fwd"

    def default_opts(self):
        return None

    def new_tape(self):
        return torch.empty(0)

    def adjoint_reset(self):
        pass

    def _mask(self, m):
        return m

    def step(self, u, p, nu, S, u_b, dt, opts, tape=None, info=False, p_prev=None, p_prev_star=None,
             p_star_out=None, u_prev=None):
        c = lambda x: None if x is None else x.detach().clone()
        self.calls.append((self.phase, c(u), c(p), c(u_prev), c(p_prev), c(p_prev_star)))
        if p_star_out is not None:
            p_star_out.copy_(p + 0.5)
        return u + 1.0 + S, 2.0 * p + 1.0

    def step_backward(self, tape, u, p, nu, u_b, dt, du1, dp1, opts=None, want=None, info=False):
        gu = du1 if du1 is not None else torch.zeros_like(u)
        gp = dp1 if dp1 is not None else torch.zeros_like(p)
        return {"u": gu.clone(), "p": gp.clone(), "S": gu.clone(), "nu": torch.zeros(1, dtype=u.dtype),
                "u_b": None if u_b is None else torch.zeros_like(u_b)}

    def outflow_update(self, u, u_b, mask, u_m, dt, out=None):
        return u_b + 0.25

    def outflow_update_backward(self, u, u_b, mask, u_m, dt, dub_out, du=None):
        return dub_out.clone(), (du if du is not None else torch.zeros_like(u))


def _expected(u0, p0, S, n, warmup=0, extrapolate=True):
    """(u, p, u_prev, p_prev, p_prev_star) of every step of the chain."""
    out, u, p, start = [], u0, p0, None
    for _ in range(warmup + n):
        out.append((u, p) + (start if start is not None else (None, None, None)))
        nxt = (u, p, p + 0.5) if extrapolate else None
        u, p, start = u + 1.0 + S, 2.0 * p + 1.0, nxt
    return out


def _same(a, b):
    return (a is None and b is None) or (a is not None and b is not None and torch.equal(a, b))


@pytest.mark.parametrize("k", [0, 2, 3])
@pytest.mark.parametrize("extrapolate", [True, False])
@pytest.mark.parametrize("warmup", [0, 2])
def test_chain_through_steps_segments_and_recompute(k, extrapolate, warmup):
    ctx = _Recorder()
    u0 = torch.arange(6, dtype=torch.float64).reshape(2, 3)
    p0 = torch.tensor([0.5, -1.0, 2.0], dtype=torch.float64)
    S = torch.full((2, 3), 0.125, dtype=torch.float64, requires_grad=True)
    nu = torch.tensor([0.01], dtype=torch.float64)
    n = 7
    uT, pT = api.rollout(ctx, u0, p0, S, nu, None, 0.1, n, checkpoint_every=k, warmup=warmup,
                         extrapolate=extrapolate)
    exp = _expected(u0, p0, S.detach(), n, warmup, extrapolate)
    fwd = [c for c in ctx.calls if c[0] == "fwd"]
    assert len(fwd) == warmup + n
    for got, want in zip(fwd, exp):
        assert all(_same(a, b) for a, b in zip(got[1:], want)), (got, want)
    ctx.phase = "bwd"
    uT.sum().backward()
    rec = [c for c in ctx.calls if c[0] == "bwd"]
    # checkpointed segments recompute their steps with the same starts (the last segment
    # first, each segment's steps in order)
    assert len(rec) == (n if k else 0)
    if k:
        segs = [exp[warmup + q:warmup + min(q + k, n)] for q in range(0, n, k)]
        order = [e for seg in reversed(segs) for e in seg]
        for got, want in zip(rec, order):
            assert all(_same(a, b) for a, b in zip(got[1:], want)), (got, want)


@pytest.mark.parametrize("k", [0, 3])
def test_chain_with_outflow(k):
    ctx = _Recorder()
    u0 = torch.ones(2, 4, dtype=torch.float64)
    p0 = torch.zeros(4, dtype=torch.float64)
    S = torch.zeros(2, 4, dtype=torch.float64)
    nu = torch.tensor([0.01], dtype=torch.float64)
    ub = torch.zeros(2, 5, dtype=torch.float64, requires_grad=True)
    api.rollout(ctx, u0, p0, S, nu, ub, 0.1, 5, checkpoint_every=k, outflow=(torch.ones(5), (1.0, 0.0)))
    exp = _expected(u0, p0, S, 5)
    fwd = [c for c in ctx.calls if c[0] == "fwd"]
    assert len(fwd) == 5
    for got, want in zip(fwd, exp):
        assert all(_same(a, b) for a, b in zip(got[1:], want))
