"""Helpers shared by the GPU tests: move seeded inputs to the device, run the oracle,
compare fields."""
import sys

import numpy as np
import torch

import cases
from oracle.piso import Geometry, step as oracle_step


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(x):
    return x.detach().double().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def rel_p(a, b):
    a = np.asarray(a) - np.mean(a)
    b = np.asarray(b) - np.mean(b)
    return rel(a, b)


def max_elem(a, b):
    """Largest element-wise difference over the largest reference magnitude: an error
    confined to a few cells (a wall row, a block seam) shows here, not in the L2 norm."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def max_elem_p(a, b):
    a = np.asarray(a) - np.mean(a)
    b = np.asarray(b) - np.mean(b)
    return max_elem(a, b)


def tight_opts(ctx, rtol_v=1e-12, rtol_p=1e-12):
    o = ctx.default_opts()
    o.vel.rtol = rtol_v
    o.pres.rtol = rtol_p
    o.pres.max_iter = 50000
    o.vel.max_iter = 2000
    return o


def random_state(case, seed, scale=0.2):
    rng = np.random.default_rng(seed)
    d, N = case.u0.shape
    u = case.u0 + scale * rng.standard_normal((d, N))
    p = rng.standard_normal(N)
    S = rng.standard_normal((d, N))
    ub = case.u_b + 0.1 * rng.standard_normal(case.u_b.shape)
    nu = case.nu * (1.0 + 0.2 * rng.random(N))
    return u, p, S, ub, nu


def two_block():
    from tests.test_oracle_pins import _two_block
    return _two_block()


def small_cases():
    return {
        "tgv16": cases.taylor_green(16, dt=0.05),
        "cavity12": cases.lid_cavity(12, n_steps=1),
        "channel": cases.channel(10, 12, 7),
        "two_block": two_block(),
        "sheared": cases.sheared_channel(9, 10, shear=0.6),
        "cylinder": cases.cylinder_oh(16, 6, 5),
        # every block with nx % 4 == 0: exercises the vectorised CG kernels
        "channel_q": cases.channel(12, 10, 8),
        "cylinder_q": cases.cylinder_oh(16, 8, 4),
    }
