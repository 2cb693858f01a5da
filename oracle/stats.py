"""FP64 oracle of the online turbulence statistics (Sec. 2.5 of the paper) and of
their gradient.

Test infrastructure: only tests, the smoke check and the benchmark's CPU baseline use
this module; the product path runs in the HIP library.

Statistics are taken over homogeneous planes of one structured block: for the planes
normal to an axis a, every plane collects the d velocity components of its cells at
every accumulated step.  Per plane the state holds the sample count n, the mean mu_i
and the central comoment sums C_ij = sum (u_i - mu_i)(u_j - mu_j) (i <= j).  A new
step contributes a batch of m samples per plane whose own mean and central sums are
taken in two passes; the batch is merged with the pairwise update for central
comoments,
    n = n_A + m,   delta = mu_B - mu_A,   mu = mu_A + delta m / n,
    C = C_A + C_B + delta_i delta_j n_A m / n,
so that no raw second moment (and its cancellation) is ever formed.  The statistics
are mean mu and covariance C / n (population form: averages over time and homogeneous
directions).

The gradient of the final mean and covariance with respect to any accumulated sample
u(P) of plane p is
    d mu_i / d u_k(P)   = delta_ik / n,
    d cov_ij / d u_k(P) = (delta_ik (u_j(P) - mu_j) + delta_jk (u_i(P) - mu_i)) / n,
because the sum of the deviations over all samples vanishes; it needs only the final
state and the sample itself, not the order of accumulation.

Parity: pinned against the definition on the concatenated samples (mean and
population covariance of all samples of a plane), order independence, exact zeros for
constant fields, shift invariance and complex-step derivatives
(tests/test_oracle_stats.py).
"""
from __future__ import annotations

import numpy as np


def pairs(d):
    """Upper-triangle component pairs (i, j), i <= j, in storage order."""
    return [(i, j) for i in range(d) for j in range(i, d)]


def plane_samples(u, dims, axis):
    """Samples of each plane normal to `axis`: array [n_planes, m, d]."""
    d = u.shape[0]
    nx, ny, nz = dims
    U = u.reshape(d, nz, ny, nx)                  # [comp, k, j, i]
    ax = {0: 3, 1: 2, 2: 1}[axis]
    U = np.moveaxis(U, ax, 1)                     # [comp, plane, ., .]
    n_planes = U.shape[1]
    return np.moveaxis(U.reshape(d, n_planes, -1), 0, 2)


def empty_state(n_planes, d):
    return {"n": 0.0, "mu": np.zeros((n_planes, d)), "C": np.zeros((n_planes, len(pairs(d))))}


def accumulate(state, u, dims, axis):
    """Merge one step's field into the state (returns a new state)."""
    X = plane_samples(u, dims, axis)              # [np, m, d]
    n_planes, m, d = X.shape
    mu_b = X.mean(axis=1)
    dev = X - mu_b[:, None, :]
    C_b = np.stack([np.sum(dev[:, :, i] * dev[:, :, j], axis=1) for i, j in pairs(d)], axis=1)
    nA = state["n"]
    n = nA + m
    delta = mu_b - state["mu"]
    mu = state["mu"] + delta * (m / n)
    corr = np.stack([delta[:, i] * delta[:, j] for i, j in pairs(d)], axis=1) * (nA * m / n)
    return {"n": n, "mu": mu, "C": state["C"] + C_b + corr}


def finalize(state):
    """(mean [np, d], covariance [np, d(d+1)/2])."""
    return state["mu"], state["C"] / state["n"]


def stats_vjp(state, u, dims, axis, mean_bar, cov_bar):
    """Gradient with respect to one accumulated field u of <mean_bar, mean> +
    <cov_bar, cov> of the final state."""
    X = plane_samples(u, dims, axis)
    n_planes, m, d = X.shape
    n, mu = state["n"], state["mu"]
    dev = X - mu[:, None, :]
    G = np.repeat(mean_bar[:, None, :] / n, m, axis=1).astype(np.result_type(X, mean_bar, cov_bar))
    for q, (i, j) in enumerate(pairs(d)):
        G[:, :, i] += cov_bar[:, q][:, None] * dev[:, :, j] / n
        G[:, :, j] += cov_bar[:, q][:, None] * dev[:, :, i] / n
    # back to the field layout
    nx, ny, nz = dims
    ax = {0: 3, 1: 2, 2: 1}[axis]
    shape = [nz, ny, nx]
    other = [s for q, s in enumerate(shape) if q != ax - 1]
    Gf = np.moveaxis(G, 2, 0).reshape(d, n_planes, *other)
    Gf = np.moveaxis(Gf, 1, ax)
    return Gf.reshape(d, -1)
