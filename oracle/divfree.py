"""FP64 oracle of the divergence-free gradient modification (Sec. 3.1 of the paper,
eq. SgradPsgrad).

Test infrastructure: only tests, the smoke check and the benchmark's CPU baseline use
this module; the product path runs in the HIP library.

For a learned source S (or velocity correction) the paper adds to the incoming
gradient dL/dS the pressure gradient lambda grad p_S of an extra pressure solve
lap p_S = div S, which is the globally consistent feedback that would make S - grad p_S
divergence free.  The discrete operators are the step's own, with A = 1:
    h = S,   rhs = div lerp(J T . h)  (no Dirichlet flux: S carries no boundary values),
    P(A = 1) p_S = rhs - mean(rhs)   (zero-mean solution, eq. pMatDiscrete with A = 1),
    g_out = dL/dS + lambda grad p_S  (central differences, p_b = p_P, as in the correction).
Then S - grad p_S has zero corrected face-flux divergence (on non-orthogonal grids the
deferred cross term is taken with a zero lagged pressure, as in a first corrector from
p = 0).

Parity: pinned by the vanishing face-flux divergence of S - grad p_S, identity at
lambda = 0 and linearity (tests/test_oracle_divfree.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .piso import Geometry, h_and_rhs, pressure_matrix, solve_pressure


def divfree_pressure(geo: Geometry, S, mode="direct", rtol=1e-13):
    N = geo.N
    A = np.ones(N)
    Pm = pressure_matrix(geo, A)
    H = sp.csr_matrix((N, N))
    zb = np.zeros((geo.d, geo.nb))
    _, rhs = h_and_rhs(geo, H, A, S, np.zeros_like(S), zb, np.zeros(N))
    return solve_pressure(Pm, rhs, mode=mode, rtol=rtol)


def divfree_gradient(geo: Geometry, S, gS, lam, mode="direct", rtol=1e-13):
    """(g_out, p_S)."""
    p = divfree_pressure(geo, S, mode, rtol)
    return gS + lam * geo.grad(p), p
