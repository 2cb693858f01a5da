"""FP64 oracle of arbitrary-order online (co)moments over homogeneous planes and of the
turbulent energy-budget terms built from them (Sec. 2.5 of the paper).

Test infrastructure: only tests, the smoke check and the benchmark's CPU baseline use
this module; the product path runs in the HIP library.

Comoments.  For m variables per sample (the d velocity components, or several fields
side by side), the central comoment sums of a set of samples are
    S_alpha = sum_s prod_i (x_si - mu_i)^alpha_i,   2 <= |alpha| <= K,
for the multi-indices alpha of total order 2 .. K.  A multi-index is written as the
sorted tuple of its variable indices (alpha = e_0 + e_2 is (0, 2)); the storage order is
by total order, then lexicographic in the tuple, so that order 2 is (0,0), (0,1), ...,
the (i <= j) pairs of the covariance.  Two sample sets A and B merge by the binomial
expansion of the deviations from the combined mean (the online formulas the paper cites
for arbitrary-order moments):
    n = n_A + n_B,  delta = mu_B - mu_A,  mu = mu_A + delta n_B / n,
    S_alpha = sum_{beta <= alpha} C(alpha, beta) [S^A_beta c_A^(alpha - beta)
                                                   + S^B_beta c_B^(alpha - beta)],
    c_A = -delta n_B / n,  c_B = delta n_A / n,
with S_0 = n_X, S_{e_i} = 0, C(alpha, beta) = prod_i binom(alpha_i, beta_i) and powers
taken per component.  The statistics are the mean and the central moments
M_alpha = S_alpha / n (population form), averaged over time and the homogeneous plane.
Their gradient with respect to one accumulated sample x_t is
    d mu_i / d x_tk = delta_ik / n,
    d M_alpha / d x_tk = (alpha_k / n) (dev_t^(alpha - e_k) - M_(alpha - e_k)),
where M of order 1 is zero and dev_t = x_t - mu (the mean's own dependence sums to the
second term).

Budget terms.  For planes normal to the axis a of a single block (the wall-normal axis
of a channel; the other axes homogeneous), with R = M of order 2 of u, the third moments
of u, the covariances G^(k) of the velocity gradients g_k = du/dx_k and the
cross-covariances X_ij = cov(u_i, dp/dx_j) over the planes:
    P_ij  = -(R_ia dU_j/dx_a + R_ja dU_i/dx_a)          production
    eps_ij = 2 sum_k G^(k)_ij                            dissipation
    T_ij  = -d <u_i' u_j' u_a'> / dx_a                   turbulent transport
    D_ij  = d^2 R_ij / dx_a^2                            viscous diffusion (as printed: no nu)
    Pi_ij = -(X_ij + X_ji)                               velocity pressure-gradient term
Readings (the paper defines the continuum terms only):
  * field gradients are cell-centred central differences in computational space mapped
    with T (d phi/dx_i = sum_j T_ji (phi_+j - phi_-j) / 2); a velocity across a Dirichlet
    face takes the ghost value 2 u_b - u_P (linear through the face value), the pressure
    takes p_b = p_P (the step's own pressure gradient, reading A7);
  * profile derivatives across the planes use the plane's metric (T_aa, J, alpha_aa =
    J T_aa^2 of its first cell; the budget is meant for grids whose metric is constant
    over each plane): d f/dx_a = T_aa (f_+ - f_-) / 2 and
    d^2 f / dx_a^2 = (1/J) [alpha_+ (f_+ - f) + alpha_- (f_- - f)] with face weights
    lerp(alpha) (the step's diffusion discretisation); across a wall the ghost is
    2 f_w - f for the first derivative and the face weight 2 alpha for the second, with
    f_w the wall value: the plane mean of u_b for U, zero for every fluctuation
    statistic; a periodic axis wraps.

Parity: pinned against the definitions on the pooled samples (loops over cells), order
independence, complex-step gradients, and closed forms of the budget terms for fields
with analytic plane statistics (tests/test_oracle_moments.py).
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np

from .piso import Geometry
from .stats import plane_samples


def multi_indices(m, K):
    """Sorted variable-index tuples of total order 2..K in storage order."""
    out = []
    for o in range(2, K + 1):
        out.extend(itertools.combinations_with_replacement(range(m), o))
    return out


def exponents(tup, m):
    e = np.zeros(m, dtype=int)
    for i in tup:
        e[i] += 1
    return e


def _dev_power(dev, e):
    """prod_i dev[..., i]^e_i over the last axis."""
    out = np.ones(dev.shape[:-1], dtype=dev.dtype)
    for i, k in enumerate(e):
        if k:
            out = out * dev[..., i] ** k
    return out


def empty_state(n_planes, m, K):
    return {"n": 0.0, "mu": np.zeros((n_planes, m)), "S": np.zeros((n_planes, len(multi_indices(m, K)))),
            "m": m, "K": K}


def _batch(X, m, K):
    """Count, mean and central sums of one batch X [np, s, m]."""
    mu = X.mean(axis=1)
    dev = X - mu[:, None, :]
    S = np.stack([_dev_power(dev, exponents(t, m)).sum(axis=1) for t in multi_indices(m, K)], axis=1)
    return X.shape[1], mu, S


def merge(nA, muA, SA, nB, muB, SB, m, K):
    """Pairwise merge of two (count, mean, central sums) sets, plane by plane."""
    idx = multi_indices(m, K)
    E = [exponents(t, m) for t in idx]
    n = nA + nB
    if nA == 0:
        return nB, muB.copy(), SB.copy()
    delta = muB - muA
    cA = -delta * (nB / n)
    cB = delta * (nA / n)

    def S_of(Sx, nx, e):
        o = int(e.sum())
        if o == 0:
            return np.full(Sx.shape[0], float(nx), dtype=Sx.dtype)
        if o == 1:
            return np.zeros(Sx.shape[0], dtype=Sx.dtype)
        return Sx[:, idx.index(tuple(i for i, k in enumerate(e) for _ in range(k)))]

    out = np.zeros((SA.shape[0], len(idx)), dtype=np.result_type(SA, SB, delta))
    for q, a in enumerate(E):
        acc = 0.0
        for b in itertools.product(*[range(k + 1) for k in a]):
            b = np.array(b)
            c = np.prod([comb(int(ai), int(bi)) for ai, bi in zip(a, b)])
            r = a - b
            acc = acc + c * (S_of(SA, nA, b) * _dev_power(cA, r) + S_of(SB, nB, b) * _dev_power(cB, r))
        out[:, q] = acc
    mu = muA + delta * (nB / n)
    return n, mu, out


def accumulate(state, x, dims, axis):
    """Merge one step's fields x [m][N] into the state (returns a new state)."""
    m, K = state["m"], state["K"]
    X = plane_samples(x, dims, axis)
    nb, mub, Sb = _batch(X, m, K)
    n, mu, S = merge(state["n"], state["mu"], state["S"], nb, mub, Sb, m, K)
    return {"n": n, "mu": mu, "S": S, "m": m, "K": K}


def finalize(state):
    """(mean [np, m], central moments [np, n_alpha])."""
    return state["mu"], state["S"] / state["n"]


def moments_vjp(state, x, dims, axis, mean_bar, mom_bar):
    """Gradient with respect to one accumulated field x of <mean_bar, mean> +
    <mom_bar, moments> of the final state."""
    m, K = state["m"], state["K"]
    idx = multi_indices(m, K)
    X = plane_samples(x, dims, axis)
    n_planes, s, _ = X.shape
    n, mu = state["n"], state["mu"]
    M = state["S"] / n
    dev = X - mu[:, None, :]
    G = np.repeat(mean_bar[:, None, :] / n, s, axis=1).astype(np.result_type(X, mean_bar, mom_bar))
    for q, t in enumerate(idx):
        a = exponents(t, m)
        for k in range(m):
            if a[k] == 0:
                continue
            r = a.copy()
            r[k] -= 1
            term = _dev_power(dev, r)
            if r.sum() >= 2:   # the lower moment; of order 1 it is zero
                term = term - M[:, idx.index(tuple(i for i, c in enumerate(r) for _ in range(c)))][:, None]
            G[:, :, k] += (a[k] / n) * mom_bar[:, q][:, None] * term
    nx, ny, nz = dims
    ax = {0: 3, 1: 2, 2: 1}[axis]
    shape = [nz, ny, nx]
    other = [sz for q, sz in enumerate(shape) if q != ax - 1]
    Gf = np.moveaxis(G, 2, 0).reshape(m, n_planes, *other)
    Gf = np.moveaxis(Gf, 1, ax)
    return Gf.reshape(m, -1)


# ------------------------------------------------------------------ budget terms

def field_gradient(geo: Geometry, phi, phi_b=None):
    """d phi_c / d x_i for every component c of phi [c][N]: [d][c][N] (axis i first).
    phi_b [c][NB]: Dirichlet face values (ghost 2 phi_b - phi_P); None: the face value
    is the cell's own (p_b = p_P)."""
    d, N = geo.d, geo.N
    nbr = geo.topo.nbr
    c = phi.shape[0]
    bface = {}
    for f in range(geo.nb):
        bface[(int(geo.bP[f]), int(geo.bj[f]), int(geo.bs[f]))] = f
    dxi = np.zeros((d, c, N), dtype=phi.dtype)
    for j in range(d):
        for P in range(N):
            vals = []
            for sd in (1, 0):
                F = nbr[P, j, sd]
                if F >= 0:
                    vals.append(phi[:, F])
                else:
                    f = bface[(P, j, sd)]
                    vals.append(2.0 * phi_b[:, f] - phi[:, P] if phi_b is not None else phi[:, P])
            dxi[j, :, P] = 0.5 * (vals[0] - vals[1])
    # d phi / d x_i = sum_j T_ji d phi / d xi_j
    return np.einsum("jin,jcn->icn", geo.T, dxi)


def _plane_metric(geo, dims, axis):
    nx, ny, nz = dims
    n = dims[axis]
    T = np.zeros(n)
    J = np.zeros(n)
    for q in range(n):
        i, j, k = [(q if a == axis else 0) for a in range(3)]
        P = i + nx * (j + ny * k)
        T[q] = geo.T[axis, axis, P]
        J[q] = geo.J[P]
    return T, J


def profile_d1(f, T, wall, periodic):
    """T (f_+ - f_-) / 2 across the planes; wall = (f at the low wall, f at the high wall)."""
    n = len(f)
    fp = np.empty_like(f)
    fm = np.empty_like(f)
    fp[:-1], fm[1:] = f[1:], f[:-1]
    if periodic:
        fp[-1], fm[0] = f[0], f[-1]
    else:
        fp[-1] = 2.0 * wall[1] - f[-1]
        fm[0] = 2.0 * wall[0] - f[0]
    return T * 0.5 * (fp - fm)


def profile_d2(f, T, J, wall, periodic):
    """(1/J) [alpha_+ (f_+ - f) + alpha_- (f_- - f)], alpha = J T^2, face weights lerp."""
    al = J * T * T
    n = len(f)
    out = np.zeros_like(f)
    for q in range(n):
        for sd in (1, -1):
            r = q + sd
            if 0 <= r < n or periodic:
                r %= n
                out[q] += 0.5 * (al[q] + al[r]) * (f[r] - f[q])
            else:
                fw = wall[1] if sd > 0 else wall[0]
                out[q] += 2.0 * al[q] * (fw - f[q])
    return out / J


def budget(geo: Geometry, dims, axis, stats_u, stats_g, stats_up, wall_mean, periodic=False):
    """Budget terms per plane for i <= j: dict of arrays [n_planes, d(d+1)/2].

    stats_u: (mean [np, d], moments [np, n_alpha]) of u with K >= 3;
    stats_g: list over k of the covariance moments [np, d(d+1)/2] of g_k = du/dx_k;
    stats_up: moments [np, n_alpha(2d, 2)] of the 2d variables (u, grad p);
    wall_mean: (U at the low wall [d], U at the high wall [d])."""
    d = geo.d
    a = axis
    T, J = _plane_metric(geo, dims, axis)
    U, Mu = stats_u
    idx_u = multi_indices(d, 3)
    idx_up = multi_indices(2 * d, 2)
    zero = (0.0, 0.0)

    def R(i, j):
        return Mu[:, idx_u.index(tuple(sorted((i, j))))]

    def T3(i, j, k):
        return Mu[:, idx_u.index(tuple(sorted((i, j, k))))]

    dU = [profile_d1(U[:, i], T, (wall_mean[0][i], wall_mean[1][i]), periodic) for i in range(d)]
    pairs = [(i, j) for i in range(d) for j in range(i, d)]
    out = {k: np.zeros((len(T), len(pairs))) for k in ("P", "eps", "T", "D", "Pi")}
    for q, (i, j) in enumerate(pairs):
        out["P"][:, q] = -(R(i, a) * dU[j] + R(j, a) * dU[i])
        out["eps"][:, q] = 2.0 * sum(Gk[:, idx_u.index((i, j))] for Gk in stats_g)
        out["T"][:, q] = -profile_d1(T3(i, j, a), T, zero, periodic)
        out["D"][:, q] = profile_d2(R(i, j), T, J, zero, periodic)
        X_ij = stats_up[:, idx_up.index((i, d + j))]
        X_ji = stats_up[:, idx_up.index((j, d + i))]
        out["Pi"][:, q] = -(X_ij + X_ji)
    return out
