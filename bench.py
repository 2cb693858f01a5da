"""Benchmark: PISO steps/s (forward and forward+adjoint) on the 96^3 turbulent-channel
workload and the pressure-CG bandwidth against the MI355X HBM roofline.

A timed step is one forward PISO step with its tape plus its adjoint step (the whole
hot path); K steps form a K-step rollout whose loss is the plane-mean statistics loss
of the channel workload, back-propagated through every step.  Inputs are resident in
HBM before the timed region.  Prints one JSON line.  The default form is MIXED (double
storage, float Krylov iterations refined to the double residual): the form that meets
1e-5 against the FP64 oracle on velocity and pressure at 96^3; the paper's FP32 form is
timed beside it for context.

    python bench.py [--gpus 1] [--steps 16] [--warmup 2] [--precision mixed|f32|f64]
                    [--workload channel96|channel192|cavity256|tgv32|cylinder5|pcg256]
                    [--no-cpu-baseline]
    python bench.py --pcg-micro 200 [--workload channel256] [--precision f32|f64|mixed] [--precond mg|jacobi]
    python bench.py --triad
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
CSRC = os.path.join(ROOT, "paper_2505_16992_amd", "csrc")
DIGEST_SOURCES = ["piso_common.h", "piso_quad.h", "piso_krylov.hip", "piso_mg.hip", "piso_line.hip",
                  "piso_zmarch.hip"]


def kernel_digest():
    """sha256 of the pressure-solver kernels' sources: counter figures recorded with a
    digest are used only while it still matches."""
    import hashlib
    h = hashlib.sha256()
    for name in DIGEST_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed counter summary, if one was
    taken for this workload with the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s_counters.md" % (kernel, workload, precision))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_digest():
        return None
    return int(vals["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_case(name):
    import cases
    if name == "channel96":
        return cases.channel(96, 96, 96)
    if name == "channel192":
        return cases.channel(192, 128, 192)
    if name == "cavity256":
        return cases.lid_cavity(256)
    if name == "tgv32":
        return cases.taylor_green(32)
    if name == "cylinder5":
        return cases.cylinder_oh()
    if name == "pcg256":
        return cases.channel(256, 256, 256)
    m = re.fullmatch(r"channel(\d+)x(\d+)x(\d+)", name) or re.fullmatch(r"channel(\d+)", name)
    if m:
        dims = [int(g) for g in m.groups()]
        return cases.channel(*(dims * 3 if len(dims) == 1 else dims))
    raise SystemExit("unknown workload " + name)


def stats_loss_grads(ctx, us, targets):
    """Channel statistics loss over a rollout (Sec. 3.2): the mean u(y) and the uv
    covariance over the homogeneous planes and the rolled-out steps, accumulated online
    by the library (piso_stats_*), against seeded target profiles.  Returns
    (L, [dL/du_n]); the gradients come from the library's statistics adjoint."""
    import torch
    u_hat, uv_hat = targets
    state = ctx.stats_state(1)
    for u in us:
        ctx.stats_accumulate(u, state, 1)
    mean, cov = ctx.stats_finalize(state, 1)
    # cov columns: (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
    ny = mean.shape[0]
    du = mean[:, 0] - u_hat
    duv = cov[:, 1] - uv_hat
    L = ((du ** 2 + duv ** 2).sum() / ny)
    mbar = torch.zeros_like(mean)
    cbar = torch.zeros_like(cov)
    mbar[:, 0] = 2.0 * du / ny
    cbar[:, 1] = 2.0 * duv / ny
    grads = [ctx.stats_backward(u, state, mbar, cbar, 1) for u in us]
    return L, grads


def _time_call(fn, reps):
    """Average ms of fn() over reps calls, HIP events on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def time_extras(ctx, case, precision, u0, S):
    """Per-call times of the calls beyond the step (the paper's outflow boundary,
    online statistics and divergence-free gradient modification)."""
    import torch
    import cases
    from paper_2505_16992_amd import api
    out = {}
    state = ctx.stats_state(1)
    out["stats_accumulate_96^3_ms"] = round(_time_call(lambda: ctx.stats_accumulate(u0, state, 1), 20), 4)
    mean, cov = ctx.stats_finalize(state, 1)
    mb, cb = torch.ones_like(mean), torch.ones_like(cov)
    du = torch.zeros_like(u0)
    out["stats_backward_96^3_ms"] = round(_time_call(lambda: ctx.stats_backward(u0, state, mb, cb, 1, du=du), 20), 4)
    g = torch.ones_like(S)
    o = ctx.default_opts().pres
    # the channel's forcing is divergence-free (its solve would see only rounding in
    # div S): a seeded perturbation gives the pressure solve a real right-hand side
    gen = torch.Generator(device=S.device).manual_seed(5)
    Sp = S + 0.1 * torch.randn(S.shape, generator=gen, device=S.device, dtype=S.dtype)
    out["divfree_gradient_96^3_ms"] = round(_time_call(lambda: ctx.divfree_gradient(Sp, g, 1.0, o), 3), 3)
    out["divfree_gradient_iters"] = ctx.divfree_gradient(Sp, g, 1.0, o, info=True)[2]["iters"]
    cyl = cases.cylinder_oh()
    cctx = api.Context(cyl.domain, precision)
    mask = cctx.outflow_mask(cases.segment_mask(cyl.domain, lambda si: cyl.domain.sides[si].block == 1))
    t = cctx.dtype
    uc = torch.as_tensor(cyl.u0, dtype=t, device="cuda")
    ub = torch.as_tensor(cyl.u_b, dtype=t, device="cuda")
    out["outflow_update_cylinder_ms"] = round(_time_call(lambda: cctx.outflow_update(uc, ub, mask, (1.0, 0.0), cyl.dt), 20), 4)
    gb = torch.ones_like(ub)
    out["outflow_update_backward_cylinder_ms"] = round(
        _time_call(lambda: cctx.outflow_update_backward(uc, ub, mask, (1.0, 0.0), cyl.dt, gb), 20), 4)
    return out


def pcg_roofline(ctx, dom, opts, tm, workload, precision):
    """(roofline, pressure_cg) records from per-class kernel times tm = {class: (ms,
    launches)}: algorithmic bytes per launch of each fine-grid kernel class (each stream
    moved once) over its average duration; the roofline names the class with the
    largest total time."""
    N, d, es = ctx.N, ctx.dim, ctx.elem_bytes
    if ctx.precision == "mixed":
        es = 4   # the inner PCG iterations of the refinement run in FP32
    mg = opts.pres.precond == 1 and bool(ctx.mg_levels)
    quad = all(b[0] % 4 == 0 for b in dom.blocks)
    nch = 2 ** d
    line = mg and bool(ctx.mg_line_axis)
    zm = mg and ctx.mg_marching_groups > 0   # plane-marching fine-grid kernels (same bytes)
    model = {
        # Pf (d), operand (z, or r and Dinv), d_old -> d_new, q
        "cg_stencil": ("k_cg_spmv_q" if quad else "k_cg_spmv", N * ((d + 4) if mg else (d + 5)) * es),
        # x, r, d_new, q, Dinv -> x, r (Jacobi)
        "cg_update": ("k_cg_update_q" if quad else "k_cg_update", N * 7 * es),
        # multigrid: x, r, d_new, q, Dinv, Pf (d) -> x, r', y, level-1 residual
        "cg_update_restrict": ("k_mg_down0uq" if quad else "k_mg_down0u", N * (d + 8) * es + (N // nch) * es),
        # r, y, Pf (d) -> level-1 residual (first V-cycle of a solve)
        "mg_down0": ("k_mg_down0", N * (d + 2) * es + (N // nch) * es),
        # y, r, Dinv, Pf (d), level-1 correction -> z
        "mg_up0": ("k_mg_up0_q" if quad else "k_mg_up0", N * (d + 4) * es + (N // nch) * es),
    }
    if zm:
        for k, name in (("cg_stencil", "k_zm_spmv"), ("cg_update_restrict", "k_zm_down"), ("mg_up0", "k_zm_up")):
            model[k] = (name, model[k][1])
    if line:
        # line smoothing: the update kernel smooths (x, r, d_new, q, Dinv, Pf along the
        # line -> x, r', y) and the restriction runs every iteration; the first
        # pre-smoothing of a solve reads r, Dinv, Pf along the line and writes y
        model["cg_update_restrict"] = ("k_line_pre", N * 9 * es)
        model["mg_smooth0"] = ("k_line_pre", N * 4 * es)
        model["mg_up0"] = ("k_line_post", N * (d + 4) * es + (N // nch) * es)
        if quad and len(dom.blocks) == 1:
            model["mg_down0"] = ("k_line_restrict", N * (d + 2) * es + (N // nch) * es)
    per = {}
    for k, (ms, n) in tm.items():
        if n:
            per[k] = {"avg_us": round(1e3 * ms / n, 3), "launches": n, "total_ms": round(ms, 3)}
            if k in model:
                per[k]["kernel"] = model[k][0]
                per[k]["bytes_per_launch"] = model[k][1]
                per[k]["GBps"] = round(model[k][1] / (ms / n * 1e-3) / 1e9, 1)
    fine = [k for k in model if k in per]
    if not fine:
        return None, None
    dom_k = max(fine, key=lambda k: per[k]["total_ms"])
    kname, kbytes = model[dom_k]
    avg = tm[dom_k][0] / tm[dom_k][1]
    ach = kbytes / (avg * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": kname, "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
            "traffic": counter_traffic(kname, workload, precision),
            "avg_launch_us": round(avg * 1e3, 3), "bytes_per_launch": kbytes,
            "launches": tm[dom_k][1]}
    iters = tm["cg_stencil"][1]
    it_ms = sum(ms for ms, _ in tm.values()) / max(iters, 1)
    it_bytes = sum(model[k][1] * tm[k][1] for k in fine) / max(iters, 1)
    pcg = {"preconditioner": "multigrid" if mg else "jacobi",
           "fine_smoother": ("lines along %s" % "xyz"[ctx.mg_line_axis]) if mg and ctx.mg_line_axis else "point",
           "mg_levels": [n for n, _ in ctx.mg_levels] if mg else [],
           "iteration_us": round(1e3 * it_ms, 3),
           "fine_bytes_per_iteration": int(it_bytes),
           "GBps": round(it_bytes / (it_ms * 1e-3) / 1e9, 1),
           "kernels": per}
    return roof, pcg


def pcg_micro(ctx, case, precision, workload, iters, precond):
    """Pressure-CG bandwidth on the pressure system of corrector 1 of step 1: a fixed
    number of PCG iterations (independent of convergence), timed as a whole and per
    kernel class, then the same system solved from p = 0 to a relative residual of 1e-8."""
    import torch
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=ctx.dtype, device="cuda")
    u0, p0, S, ub = dev(case.u0), dev(case.p0), dev(case.S), dev(case.u_b)
    nu = dev(np.array([case.nu]))
    opts = ctx.default_opts()
    opts.pres.precond = precond
    sys_ = ctx.new_system()
    ctx.assemble(sys_, u0, p0, nu, S, ub, case.dt)
    us = u0.clone()
    ctx.solve_velocity(sys_, us, opts.vel)
    fixed = type(opts.pres)()
    fixed.rtol, fixed.max_iter, fixed.check_every, fixed.precond = 1e-30, iters, iters, precond
    fixed.inner_rtol, fixed.max_refine = 1e-30, 0
    p = torch.zeros_like(p0)
    out = {"mode": "pcg_micro", "workload": workload, "cells": ctx.N, "precision": precision,
           "preconditioner": "multigrid" if precond == 1 else "jacobi"}
    if precision != "mixed":
        ctx.solve_pressure(sys_, us, ub, p0, p, fixed)     # warm-up (graph recording, setup)
        torch.cuda.synchronize()
        reps = 3
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            p.zero_()
            inf = ctx.solve_pressure(sys_, us, ub, p0, p, fixed)
        b.record()
        torch.cuda.synchronize()
        out["fixed_iters"] = inf["iters"]
        out["fixed_solve_ms"] = round(a.elapsed_time(b) / reps, 4)
        ctx.set_timing(True)
        p.zero_()
        ctx.solve_pressure(sys_, us, ub, p0, p, fixed)
        torch.cuda.synchronize()
        tm = ctx.get_timing()
        ctx.set_timing(False)
        roof, pcg = pcg_roofline(ctx, case.domain, opts, tm, workload, precision)
        out["roofline"], out["pressure_cg"] = roof, pcg
    # to the equal-residual target 1e-8 from p = 0 (F32: to its own default 1e-6; the
    # float recurrence does not reach 1e-8)
    tol = type(opts.pres)()
    goal = 1e-6 if precision == "f32" else 1e-8
    tol.rtol, tol.max_iter, tol.check_every, tol.precond = goal, 2000, 4, precond
    tol.inner_rtol, tol.max_refine = opts.pres.inner_rtol, opts.pres.max_refine
    p.zero_()
    ctx.solve_pressure(sys_, us, ub, p0, p, tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.zero_()
    inf = ctx.solve_pressure(sys_, us, ub, p0, p, tol)
    torch.cuda.synchronize()
    out["solve_to_rtol"] = {"rtol": goal, "ms": round(1e3 * (time.perf_counter() - t0), 3), "iters": inf["iters"],
                         "refinements": inf["refinements"], "rel_residual": inf["rel_residual"]}
    return out


def stream_triad(gib=4.0, reps=20):
    """STREAM-type triad a = b + s c on float32 arrays of `gib` GiB each (torch's
    elementwise kernel): the achievable HBM ceiling beside the 8 TB/s peak."""
    import torch
    n = int(gib * (1 << 30)) // 4
    b = torch.ones(n, dtype=torch.float32, device="cuda")
    c = torch.ones(n, dtype=torch.float32, device="cuda")
    a = torch.empty_like(b)
    torch.add(b, c, alpha=3.0, out=a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(b, c, alpha=3.0, out=a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"mode": "stream_triad", "bytes_per_call": 3 * n * 4, "ms": round(ms, 4),
            "GBps": round(3 * n * 4 / (ms * 1e-3) / 1e9, 1)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, precision):
    """The FP64 oracle, as it stands, on this host: one forward PISO step of the same
    workload from the same initial state, then that step's adjoint for the gradient of
    <1, u^{n+1}> (iterative solves at rtol 1e-10 in 3D, direct in 2D).  Threads used =
    process CPU time / wall time of the sample."""
    from oracle.adjoint import step_vjp
    from oracle.piso import Geometry, step as oracle_step
    dom = case.domain
    mode = "iterative" if dom.dim == 3 else "direct"
    geo = Geometry(dom)
    up = case.u0.astype(np.float32).astype(np.float64) if precision == "f32" else case.u0
    w0, c0 = time.perf_counter(), time.process_time()
    rec = oracle_step(geo, up, case.p0, case.nu, case.S, case.dt, case.u_b, mode=mode, rtol=1e-10)
    w1, c1 = time.perf_counter(), time.process_time()
    step_vjp(geo, rec, np.ones_like(up), np.zeros(geo.N), mode=mode, rtol=1e-10)
    w2, c2 = time.perf_counter(), time.process_time()
    fwd, adj = w1 - w0, w2 - w1
    used = (c2 - c0) / max(w2 - w0, 1e-9)
    env = {k: os.environ.get(k, "") for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    return {"value": round(1.0 / (fwd + adj), 5), "unit": "fwd+adjoint steps/s",
            "cores": max(1, int(round(used))), "kind": "oracle",
            "fwd_steps_per_s": round(1.0 / fwd, 5),
            "sample": "one forward PISO step of the same workload and its adjoint (FP64 oracle, %s solves at "
                      "rtol 1e-10): forward %.1f s, adjoint %.1f s; CPU time / wall time %.2f; host: %s, "
                      "%d logical cores; thread environment %s"
                      % (mode, fwd, adj, used, _cpu_model(), os.cpu_count(), env)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="mixed", choices=["f32", "mixed", "f64"])
    ap.add_argument("--workload", default="channel96")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32-context", action="store_true",
                    help="skip the FP32-form figures reported beside a MIXED run")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the per-call timings of the outflow, statistics and gradient-modification calls")
    ap.add_argument("--kernel-digest", action="store_true", help="print the CG kernel source digest")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 256 MiB (counter calibration)")
    ap.add_argument("--pcg-micro", type=int, default=0, metavar="ITERS",
                    help="only the pressure-CG microbenchmark: ITERS fixed PCG iterations on the "
                         "corrector-1 system of step 1, then the same system solved to 1e-8")
    ap.add_argument("--precond", default="mg", choices=["mg", "jacobi"],
                    help="pressure preconditioner of --pcg-micro")
    ap.add_argument("--triad", action="store_true", help="only the STREAM-type triad ceiling")
    ap.add_argument("--pres-rtol", type=float, default=None,
                    help="pressure tolerance (equal-residual comparisons of the precision forms)")
    args = ap.parse_args()

    if args.kernel_digest:
        print(kernel_digest())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the PISO step here runs on a single MI355X "
              "(multi-GPU sharding is described in DESIGN.md, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import cases
    from paper_2505_16992_amd import api

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # one elementwise kernel that reads 256 MiB and writes 256 MiB
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.add(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"read_bytes": x.numel() * 4, "write_bytes": y.numel() * 4}}))
        return
    if args.triad:
        print(json.dumps(stream_triad()), flush=True)
        return
    case = make_case(args.workload)
    dom = case.domain
    ctx = api.Context(dom, args.precision)
    if args.pcg_micro:
        print(json.dumps(pcg_micro(ctx, case, args.precision, args.workload, args.pcg_micro,
                                   1 if args.precond == "mg" else 0)), flush=True)
        return
    N, d = ctx.N, ctx.dim
    log("workload %s N=%d precision %s dt=%.3e" % (args.workload, N, args.precision, case.dt))
    K, W = args.steps, args.warmup
    is_channel = args.workload.startswith("channel") or args.workload == "pcg256"
    targets = None
    if is_channel:
        u_hat, uv_hat = cases.channel_loss_targets(case)
        targets = (torch.as_tensor(u_hat, dtype=torch.float64, device="cuda"),
                   torch.as_tensor(uv_hat, dtype=torch.float64, device="cuda"))

    def runner(cx):
        """(fwd_adj, fwd, opts, S) for context cx: the workload's inputs in its precision."""
        def dev(x):
            return torch.as_tensor(np.ascontiguousarray(x), dtype=cx.dtype, device="cuda")

        u0, p0, S, ub = dev(case.u0), dev(case.p0), dev(case.S), dev(case.u_b)
        nu = dev(np.array([case.nu]))
        opts = cx.default_opts()
        if args.pres_rtol is not None:
            opts.pres.rtol = args.pres_rtol

        def fwd_adj(n_steps):
            """n-step rollout with tapes, then its adjoint; returns (dS, info)."""
            us, ps, tapes = [u0], [p0], []
            infos = []
            pst = None
            for _ in range(n_steps):
                t = cx.new_tape()
                # the linear solves start from the previous step's fields (piso_step_opts)
                uv, pv, pvs, pst = ((us[-2], ps[-2]) if len(ps) > 1 else (None, None)) + (pst, torch.empty_like(p0))
                u1, p1, inf = cx.step(us[-1], ps[-1], nu, S, ub, case.dt, opts, tape=t, info=True, p_prev=pv,
                                      p_prev_star=pvs, p_star_out=pst, u_prev=uv)
                us.append(u1)
                ps.append(p1)
                tapes.append(t)
                infos.append(inf)
            if is_channel:
                _, gus = stats_loss_grads(cx, us[1:], targets)
            else:
                gus = [torch.zeros_like(u0) for _ in range(n_steps)]
                gus[-1] = torch.ones_like(u0)
            dS = torch.zeros_like(S)
            gu, gp = None, None
            cx.adjoint_reset()   # adjoint pressure solves warm-start within this rollout only
            for q in range(n_steps - 1, -1, -1):
                gin = gus[q] if gu is None else gus[q] + gu
                g = cx.step_backward(tapes[q], us[q], ps[q], nu, ub, case.dt, gin, gp, opts, want=("u", "p", "S"))
                gu, gp = g["u"], g["p"]
                dS += g["S"]
                tapes[q] = None
            return dS, infos

        def fwd(n_steps):
            u, p, uv, pv, pvs = u0, p0, None, None, None
            infos = []
            for _ in range(n_steps):
                pst = torch.empty_like(p0)
                u1, p1, inf = cx.step(u, p, nu, S, ub, case.dt, opts, info=True, p_prev=pv, p_prev_star=pvs,
                                      p_star_out=pst, u_prev=uv)
                uv, pv, pvs, u, p = u, p, pst, u1, p1
                infos.append(inf)
            return infos

        return fwd_adj, fwd, opts, (u0, S)

    fwd_adj, fwd, opts, (u0, S) = runner(ctx)

    # warm-up (untimed)
    if W:
        fwd_adj(W)
    torch.cuda.synchronize()

    # timed region: K forward+adjoint steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dS, infos = fwd_adj(K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T = t1 - t0
    # forward-only rollout, timed separately
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    finfos = fwd(K)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    Tf = t3 - t2
    cg_iters = [sum(i["pres"][k]["iters"] for k in range(2)) for i in finfos]
    bi_iters = [i["vel"]["iters"] for i in finfos]
    log("fwd+adj %.3f s (%d steps), fwd %.3f s; CG iters/step %s; BiCGStab iters/step %s"
        % (T, K, Tf, cg_iters, bi_iters))

    roof = None
    pcg = None
    if not args.no_roofline:
        # roofline pass: same forward+adjoint workload with HIP events around every
        # pressure-CG kernel launch (on the library's stream)
        ctx.set_timing(True)
        fwd_adj(K)
        torch.cuda.synchronize()
        tm = ctx.get_timing()
        ctx.set_timing(False)
        roof, pcg = pcg_roofline(ctx, dom, opts, tm, args.workload, args.precision)
        log("timing %s" % tm)

    # the paper's own FP32 form on the same workload, for context (its pressure at 96^3 is
    # 4.7e-5 from the FP64 oracle, beyond the 1e-5 the MIXED form meets)
    f32_ctx = None
    if args.precision == "mixed" and not args.no_f32_context:
        cx = api.Context(dom, "f32")
        fa, fw, o32, _ = runner(cx)
        if W:
            fa(W)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        fa(K)
        torch.cuda.synchronize()
        a1 = time.perf_counter()
        fw(K)
        torch.cuda.synchronize()
        a2 = time.perf_counter()
        f32_ctx = {"fwd_adj_steps_per_s": round(K / (a1 - a0), 4), "fwd_steps_per_s": round(K / (a2 - a1), 4),
                   "pres_rtol": o32.pres.rtol}
        log("f32 context %s" % f32_ctx)
        del cx

    extras = None
    if not args.no_extras and args.workload == "channel96":
        extras = time_extras(ctx, case, args.precision, u0, S)
        log("extras %s" % extras)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case, args.precision)
        log("cpu baseline %s" % cpu)

    out = {
        "metric": "PISO steps/s fwd and fwd+adjoint at 96^3 channel; pressure-CG HBM GB/s",
        "value": round(K / T, 4),
        "unit": "fwd+adjoint steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(1e3 * T / K, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "mixed": "f32+f64", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": N, "dt": case.dt, "precision": args.precision,
                   "rollout_steps": K, "pres_rtol": opts.pres.rtol, "vel_rtol": opts.vel.rtol},
        "pres_rel_residual_last": finfos[-1]["pres"][1]["rel_residual"],
        "fwd_steps_per_s": round(K / Tf, 4),
        "cell_updates_per_s_fwd": round(N * K / Tf, 1),
        "cell_updates_per_s_fwd_adj": round(N * K / T, 1),
        "cg_iters_per_fwd_step": float(np.mean(cg_iters)),
        "bicgstab_iters_per_fwd_step": float(np.mean(bi_iters)),
        "pressure_cg": pcg,
        "roofline": roof,
        "cpu_baseline": cpu,
        "f32_form": f32_ctx,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
