"""Plane-marching fine-grid kernels of the multigrid PCG (3D grids whose blocks have
nx % 4 == 0, point smoothing on the fine level) against the oracle's direct solves.

The kernels compute the same PCG iteration as the one-quad-per-thread kernels in another
summation order, so the checks are the oracle's step and step adjoint to solver
tolerance.  Small tilings (PISO_ZM_TILE="xq,rt,ks") put tile edges in x and y and run
ends in z everywhere on small grids, so that every path is taken: neighbours from LDS,
from the rows beside the tile, from the planes beyond the run, across periodic sides of
the block and across sides connected to other blocks, and the one-row and one-plane
aggregates of odd extents.
"""
import numpy as np
import pytest
import torch

import cases
from oracle.adjoint import step_vjp
from oracle.piso import Geometry, step as oracle_step
from tests.gpu_common import dev, host, max_elem, random_state, rel, rel_p, say, small_cases, tight_opts

pytestmark = pytest.mark.gpu

MG = 1


def _api():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2505_16992_amd import api
    return api


def blocks4():
    """Four 8x6x4 blocks in a 2x2 arrangement in (y, z): sides in y and z connect blocks
    (z through the pairs periodically), x wraps onto each block, walls at the outer y
    sides; y stretched differently in the two block rows."""
    xv = np.linspace(0.0, 1.0, 9)
    y_lo = cases.tanh_vertices(6, 1.2, 0.0, 0.5)
    y_hi = np.linspace(0.5, 1.0, 7)
    z_lo, z_hi = np.linspace(0.0, 0.4, 5), np.linspace(0.4, 1.0, 5)
    parts = [cases.tensor_metrics([xv, yv, zv]) for zv in (z_lo, z_hi) for yv in (y_lo, y_hi)]
    T, J, c = cases.concat_blocks(parts)
    S_ = cases.Side
    sides = []
    for b in range(4):
        sides += cases.periodic_sides(b, 3, (0,))
    # block b = 2 * (z row) + (y row)
    sides += [S_(0, 3, cases.CONNECT, other_block=1), S_(1, 2, cases.CONNECT, other_block=0),
              S_(2, 3, cases.CONNECT, other_block=3), S_(3, 2, cases.CONNECT, other_block=2),
              S_(0, 5, cases.CONNECT, other_block=2), S_(2, 4, cases.CONNECT, other_block=0),
              S_(1, 5, cases.CONNECT, other_block=3), S_(3, 4, cases.CONNECT, other_block=1),
              S_(2, 5, cases.CONNECT, other_block=0), S_(0, 4, cases.CONNECT, other_block=2),
              S_(3, 5, cases.CONNECT, other_block=1), S_(1, 4, cases.CONNECT, other_block=3),
              S_(0, 2, cases.DIRICHLET), S_(2, 2, cases.DIRICHLET),
              S_(1, 3, cases.DIRICHLET), S_(3, 3, cases.DIRICHLET)]
    dom = cases.Domain(3, [(8, 6, 4)] * 4, sides, T, J, c)
    N = dom.n_cells
    ub = cases.boundary_values(dom, lambda si: np.array([0.5, 0.0, 0.1]) if dom.sides[si].side == 3
                               else np.zeros(3))
    return cases.Case("blocks4", dom, np.zeros((3, N)), np.zeros(N), np.zeros((3, N)), 0.02, 0.05, ub, 1)


def blocks2_unequal():
    """Two blocks of different x extents (8 and 12 cells) side by side along x, periodic in x
    through the pair, walls in y, z wrapping onto each block: tiles of different widths."""
    y = cases.tanh_vertices(6, 1.1, 0.0, 1.0)
    z = np.linspace(0.0, 0.5, 5)
    parts = [cases.tensor_metrics([np.linspace(0.0, 0.8, 9), y, z]),
             cases.tensor_metrics([np.linspace(0.8, 2.0, 13), y, z])]
    T, J, c = cases.concat_blocks(parts)
    S_ = cases.Side
    sides = [S_(0, 1, cases.CONNECT, other_block=1), S_(1, 0, cases.CONNECT, other_block=0),
             S_(1, 1, cases.CONNECT, other_block=0), S_(0, 0, cases.CONNECT, other_block=1)]
    for b in range(2):
        sides += cases.periodic_sides(b, 3, (2,)) + [S_(b, 2, cases.DIRICHLET), S_(b, 3, cases.DIRICHLET)]
    dom = cases.Domain(3, [(8, 6, 4), (12, 6, 4)], sides, T, J, c)
    N = dom.n_cells
    ub = cases.boundary_values(dom, lambda si: np.array([0.4, 0.0, -0.2]) if dom.sides[si].side == 3
                               else np.zeros(3))
    return cases.Case("blocks2", dom, np.zeros((3, N)), np.zeros(N), np.zeros((3, N)), 0.02, 0.05, ub, 1)


def periodic_box():
    """One 8x6x6 block, every side wrapping onto the block, mildly stretched in y."""
    xv = np.linspace(0.0, 1.0, 9)
    yv = np.cumsum(np.r_[0.0, 0.12, 0.15, 0.2, 0.2, 0.18, 0.15])
    zv = np.linspace(0.0, 0.8, 7)
    T, J, c = cases.tensor_metrics([xv, yv, zv])
    dom = cases.Domain(3, [(8, 6, 6)], cases.periodic_sides(0, 3, (0, 1, 2)), T, J, c)
    N = dom.n_cells
    return cases.Case("box", dom, np.zeros((3, N)), np.zeros(N), np.zeros((3, N)), 0.03, 0.05,
                      np.zeros((3, 0)), 1)


def zm_cases():
    return {
        "channel_q": small_cases()["channel_q"],        # 12 x 10 x 8, walls in y
        "channel_odd": cases.channel(8, 7, 9),          # odd ny and nz: one-row and one-plane aggregates
        "blocks4": blocks4(),
        "blocks2": blocks2_unequal(),
        "box": periodic_box(),
    }


# default tiles (whole rows, one tile in y on these grids); tiles of one quad by two rows
# through two planes; two quads by four rows through four planes
TILES = [None, "1,2,2", "2,4,4"]


def _ctx(api, case, prec, tile, monkeypatch):
    monkeypatch.setenv("PISO_MG_LINE", "0")
    monkeypatch.setenv("PISO_ZMARCH", "1")   # these grids are below the size the kernels start at
    if tile:
        monkeypatch.setenv("PISO_ZM_TILE", tile)
    ctx = api.Context(case.domain, prec)
    monkeypatch.delenv("PISO_ZM_TILE", raising=False)
    monkeypatch.delenv("PISO_ZMARCH")
    monkeypatch.delenv("PISO_MG_LINE")
    assert ctx.mg_line_axis == 0 and ctx.mg_marching_groups > 0
    return ctx


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("name", list(zm_cases()))
def test_zmarch_step_and_adjoint_f64(name, tile, monkeypatch):
    """One FP64 step and its adjoint with the multigrid PCG against the oracle (direct
    solves) to solver tolerance, element by element."""
    api = _api()
    case = zm_cases()[name]
    say("test_zmarch_step_and_adjoint_f64", name, tile)
    u, p, S, ub, nu = random_state(case, seed=61)
    geo = Geometry(case.domain)
    ref = oracle_step(geo, u, p, nu, S, case.dt, ub)
    rng = np.random.default_rng(62)
    w = rng.standard_normal(u.shape)
    gr = step_vjp(geo, ref, w, np.zeros(geo.N))
    ctx = _ctx(api, case, "f64", tile, monkeypatch)
    t = ctx.dtype
    o = tight_opts(ctx)
    assert o.pres.precond == MG
    args = [dev(x, t) for x in (u, p, nu, S, ub)]
    tape = ctx.new_tape()
    u1, p1, info = ctx.step(*args, case.dt, o, tape=tape, info=True)
    g = ctx.step_backward(tape, args[0], args[1], args[2], args[4], case.dt, dev(w, t), None, o)
    eu, ep = max_elem(host(u1), ref.u2), rel_p(host(p1), ref.p2)
    eg = max(max_elem(host(g["S"]), gr["S"]), max_elem(host(g["u"]), gr["u_n"]))
    say("  %d groups, iters %s: max elem u %.2e, rel p %.2e, max elem grad %.2e" % (
        ctx.mg_marching_groups, [q["iters"] for q in info["pres"]], eu, ep, eg))
    assert all(q["status"] == 0 for q in info["pres"])
    assert eu < 1e-9 and ep < 1e-8 and eg < 1e-8


@pytest.mark.parametrize("prec", ["f32", "mixed"])
@pytest.mark.parametrize("tile", [None, "1,2,2"])
def test_zmarch_single_precision(prec, tile, monkeypatch):
    api = _api()
    for name, case in zm_cases().items():
        u, p, S, ub, nu = random_state(case, seed=63)
        ref = oracle_step(Geometry(case.domain), u, p, nu, S, case.dt, ub)
        ctx = _ctx(api, case, prec, tile, monkeypatch)
        t = ctx.dtype
        o = ctx.default_opts()
        u1, p1, info = ctx.step(dev(u, t), dev(p, t), dev(nu, t), dev(S, t), dev(ub, t), case.dt, o, info=True)
        eu, ep = rel(host(u1), ref.u2), rel_p(host(p1), ref.p2)
        say("%s %s %s: iters %s, rel err u %.2e p %.2e" % (name, prec, tile, [q["iters"] for q in info["pres"]],
                                                         eu, ep))
        assert all(q["status"] == 0 for q in info["pres"])
        assert eu < (1e-8 if prec == "mixed" else 1e-5) and ep < (1e-7 if prec == "mixed" else 1e-5)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_zmarch_matches_quad_kernels(prec, monkeypatch):
    """Against the one-quad-per-thread kernels (PISO_ZMARCH=0) on the same system: the
    same solution to solver tolerance and iteration counts within one."""
    api = _api()
    case = cases.channel(16, 12, 10)
    u, p, S, ub, nu = random_state(case, seed=64)
    out = []
    for env in ("1", "0"):
        monkeypatch.setenv("PISO_MG_LINE", "0")
        monkeypatch.setenv("PISO_ZMARCH", env)
        ctx = api.Context(case.domain, prec)
        monkeypatch.delenv("PISO_ZMARCH")
        assert (ctx.mg_marching_groups > 0) == (env == "1")
        t = ctx.dtype
        o = tight_opts(ctx) if prec == "f64" else ctx.default_opts()
        u1, p1, info = ctx.step(dev(u, t), dev(p, t), dev(nu, t), dev(S, t), dev(ub, t), case.dt, o, info=True)
        out.append((host(u1), host(p1), [q["iters"] for q in info["pres"]]))
    (ua, pa, ia), (ub_, pb, ib) = out
    say("%s: iterations marching %s, per-quad %s; rel u %.2e p %.2e" % (prec, ia, ib, rel(ua, ub_), rel_p(pa, pb)))
    assert all(abs(a - b) <= 1 for a, b in zip(ia, ib))
    tol = 1e-10 if prec == "f64" else 1e-5
    assert rel(ua, ub_) < tol and rel_p(pa, pb) < tol


def _plain_channel(nx, ny, nz):
    """The channel's block layout and metrics without its initial field (cheap to build)."""
    T, J, c = cases.tensor_metrics([np.linspace(0.0, 6.0, nx + 1), cases.tanh_vertices(ny, 1.5, -1.0, 1.0),
                                    np.linspace(0.0, 3.0, nz + 1)])
    sides = cases.periodic_sides(0, 3, (0, 2)) + [cases.Side(0, 2, cases.DIRICHLET), cases.Side(0, 3, cases.DIRICHLET)]
    return cases.Domain(3, [(nx, ny, nz)], sides, T, J, c)


def test_zmarch_size_rule(monkeypatch):
    """Without PISO_ZMARCH the marching kernels run only where a field of the pressure
    Krylov vectors takes 8 MiB: 128^3 in float (exactly 8 MiB) and 192x128x192, not 96^3
    (7.1 MB in double, 3.5 MB in float)."""
    api = _api()
    monkeypatch.setenv("PISO_MG_LINE", "0")
    for dims, prec, on in (((96, 96, 96), "f64", False), ((96, 96, 96), "f32", False),
                           ((128, 128, 128), "mixed", True), ((192, 128, 192), "f32", True)):
        ctx = api.Context(_plain_channel(*dims), prec)
        say("%s %s: marching groups %d" % (dims, prec, ctx.mg_marching_groups))
        assert (ctx.mg_marching_groups > 0) == on
        del ctx


def test_zmarch_graph_replay_and_determinism(monkeypatch):
    """Replays of the recorded PCG pair give bit-identical steps to eager launches, and two
    contexts give bit-identical results (fixed summation order)."""
    api = _api()
    case = zm_cases()["blocks4"]
    u, p, S, ub, nu = random_state(case, seed=65)
    res = []
    for graphs in ("1", "0", "0"):
        monkeypatch.setenv("PISO_NO_GRAPH", graphs)
        ctx = _ctx(api, case, "f32", "2,4,4", monkeypatch)
        monkeypatch.delenv("PISO_NO_GRAPH")
        t = ctx.dtype
        o = ctx.default_opts()
        uu, pp = dev(u, t), dev(p, t)
        seq = []
        for _ in range(3):
            uu, pp = ctx.step(uu, pp, dev(nu, t), dev(S, t), dev(ub, t), case.dt, o)
            torch.cuda.synchronize()
            seq.append((uu.clone(), pp.clone()))
        res.append(seq)
    for a, b, c in zip(*res):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        assert torch.equal(b[0], c[0]) and torch.equal(b[1], c[1])
