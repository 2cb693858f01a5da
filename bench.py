"""Benchmark: PISO steps/s (forward and forward+adjoint) on the 96^3 turbulent-channel
workload and the pressure-CG bandwidth against the MI355X HBM roofline.

A timed step is one forward PISO step with its tape plus its adjoint step (the whole
hot path); K steps form a K-step rollout whose loss is the plane-mean statistics loss
of the channel workload, back-propagated through every step.  Inputs are resident in
HBM before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 16] [--warmup 2] [--precision f32|mixed|f64]
                    [--workload channel96|channel192|cavity256|tgv32|cylinder5|pcg256]
                    [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
CSRC = os.path.join(ROOT, "paper_2505_16992_amd", "csrc")
DIGEST_SOURCES = ["piso_common.h", "piso_quad.h", "piso_krylov.hip", "piso_mg.hip"]


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
    raise SystemExit("unknown workload " + name)


def stats_loss_grads(us, y_planes, targets, nx, ny, nz):
    """Channel statistics loss over a rollout: plane means of u and of the uv
    covariance, averaged over the steps, against seeded target profiles.  Returns
    (L, [dL/du_n])."""
    import torch
    u_hat, uv_hat = targets
    leaves = [u.detach().requires_grad_(True) for u in us]
    ubar = 0.0
    uv = 0.0
    for u in leaves:
        U = u[0].reshape(nz, ny, nx)
        V = u[1].reshape(nz, ny, nx)
        mu = U.mean(dim=(0, 2))
        mv = V.mean(dim=(0, 2))
        ubar = ubar + mu
        uv = uv + (U * V).mean(dim=(0, 2)) - mu * mv
    ubar = ubar / len(leaves)
    uv = uv / len(leaves)
    L = ((ubar - u_hat) ** 2 + (uv - uv_hat) ** 2).mean()
    grads = torch.autograd.grad(L, leaves)
    return L.detach(), [g.contiguous() for g in grads]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f32", choices=["f32", "mixed", "f64"])
    ap.add_argument("--workload", default="channel96")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--kernel-digest", action="store_true", help="print the CG kernel source digest")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 256 MiB (counter calibration)")
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
    case = make_case(args.workload)
    dom = case.domain
    ctx = api.Context(dom, args.precision)
    dt_t = ctx.dtype
    N, d = ctx.N, ctx.dim
    log("workload %s N=%d precision %s dt=%.3e" % (args.workload, N, args.precision, case.dt))

    def dev(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=dt_t, device="cuda")

    u0, p0, S, ub = dev(case.u0), dev(case.p0), dev(case.S), dev(case.u_b)
    nu = dev(np.array([case.nu]))
    opts = ctx.default_opts()
    if args.pres_rtol is not None:
        opts.pres.rtol = args.pres_rtol
    K, W = args.steps, args.warmup
    is_channel = args.workload.startswith("channel") or args.workload == "pcg256"
    if is_channel:
        nx, ny, nz = dom.blocks[0]
        u_hat, uv_hat = cases.channel_loss_targets(case)
        targets = (dev(u_hat), dev(uv_hat))

    def fwd_adj(n_steps):
        """n-step rollout with tapes, then its adjoint; returns (dS, info)."""
        us, ps, tapes = [u0], [p0], []
        infos = []
        for _ in range(n_steps):
            t = ctx.new_tape()
            u1, p1, inf = ctx.step(us[-1], ps[-1], nu, S, ub, case.dt, opts, tape=t, info=True)
            us.append(u1)
            ps.append(p1)
            tapes.append(t)
            infos.append(inf)
        if is_channel:
            _, gus = stats_loss_grads(us[1:], None, targets, nx, ny, nz)
        else:
            gus = [torch.zeros_like(u0) for _ in range(n_steps)]
            gus[-1] = torch.ones_like(u0)
        dS = torch.zeros_like(S)
        gu, gp = None, None
        for q in range(n_steps - 1, -1, -1):
            gin = gus[q] if gu is None else gus[q] + gu
            g = ctx.step_backward(tapes[q], us[q], ps[q], nu, ub, case.dt, gin, gp, opts, want=("u", "p", "S"))
            gu, gp = g["u"], g["p"]
            dS += g["S"]
            tapes[q] = None
        return dS, infos

    def fwd(n_steps):
        u, p = u0, p0
        infos = []
        for _ in range(n_steps):
            u, p, inf = ctx.step(u, p, nu, S, ub, case.dt, opts, info=True)
            infos.append(inf)
        return infos

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
        es = ctx.elem_bytes
        mg = opts.pres.precond == 1 and bool(ctx.mg_levels)
        quad = all(b[0] % 4 == 0 for b in dom.blocks)
        nch = 2 ** d
        # algorithmic bytes per launch of each fine-grid kernel class (each stream once)
        model = {
            # Pf (d), operand (z, or r and Dinv), d_old -> d_new, q
            "cg_stencil": ("k_cg_spmv_q" if quad else "k_cg_spmv", N * ((d + 4) if mg else (d + 5)) * es),
            # x, r, d_new, q, Dinv -> x, r (+ y = omega Dinv r for the multigrid)
            "cg_update": ("k_cg_update_q" if quad else "k_cg_update", N * (8 if mg else 7) * es),
            # r, y, Pf (d) -> level-1 residual
            "mg_down0": ("k_mg_down0", N * (d + 2) * es + (N // nch) * es),
            # y, r, Dinv, Pf (d), level-1 correction -> z
            "mg_up0": ("k_mg_up0_q" if quad else "k_mg_up0", N * (d + 4) * es + (N // nch) * es),
        }
        per = {}
        for k, (ms, n) in tm.items():
            if n:
                per[k] = {"avg_us": round(1e3 * ms / n, 3), "launches": n, "total_ms": round(ms, 3)}
                if k in model:
                    per[k]["kernel"] = model[k][0]
                    per[k]["bytes_per_launch"] = model[k][1]
                    per[k]["GBps"] = round(model[k][1] / (ms / n * 1e-3) / 1e9, 1)
        fine = [k for k in model if k in per]
        if fine:
            dom_k = max(fine, key=lambda k: per[k]["total_ms"])
            kname, kbytes = model[dom_k]
            avg = tm[dom_k][0] / tm[dom_k][1]
            ach = kbytes / (avg * 1e-3) / 1e9
            roof = {"bound": "hbm", "kernel": kname, "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
                    "traffic": counter_traffic(kname, args.workload, args.precision),
                    "avg_launch_us": round(avg * 1e3, 3), "bytes_per_launch": kbytes,
                    "launches": tm[dom_k][1]}
            iters = tm["cg_stencil"][1]
            it_ms = sum(ms for ms, _ in tm.values()) / max(iters, 1)
            it_bytes = sum(model[k][1] * tm[k][1] for k in fine) / max(iters, 1)
            pcg = {"preconditioner": "multigrid" if mg else "jacobi",
                   "mg_levels": [n for n, _ in ctx.mg_levels] if mg else [],
                   "iteration_us": round(1e3 * it_ms, 3),
                   "fine_bytes_per_iteration": int(it_bytes),
                   "GBps": round(it_bytes / (it_ms * 1e-3) / 1e9, 1),
                   "kernels": per}
        log("timing %s" % tm)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle.piso import Geometry, step as oracle_step
        geo = Geometry(dom)
        up = case.u0.astype(np.float32).astype(np.float64) if args.precision != "f64" else case.u0
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        tc0 = time.perf_counter()
        oracle_step(geo, up, case.p0, case.nu, case.S, case.dt, case.u_b,
                    mode="iterative" if d == 3 else "direct", rtol=1e-10)
        tc = time.perf_counter() - tc0
        cpu = {"value": round(1.0 / tc, 5), "unit": "fwd steps/s", "cores": 1, "kind": "oracle",
               "sample": "one forward PISO step of the same workload (FP64 oracle, %s solves at rtol 1e-10): %.1f s; "
                         "SciPy sparse kernels run single-threaded, host has %d cores"
                         % ("iterative" if d == 3 else "direct", tc, os.cpu_count())}
        log("cpu baseline %.1f s" % tc)

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
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
