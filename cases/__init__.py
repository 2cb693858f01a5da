"""Seeded synthetic inputs for the multi-block PISO step.

This module only *generates inputs*: block layouts, vertex meshes, the cell-centre
transformation metrics T and J that the method takes as given (Sec. 2.2 and
App. A.3.2 of the paper: T_ji = d xi^j / d x_i at cell centres, J = det(T^-1)),
initial fields, sources, boundary values, time steps and seeds.  It contains none of
the method's own arithmetic (no fluxes, matrices, solves or corrections), so both the
CPU oracle and the HIP library may consume what it produces.

Conventions shared with the C-ABI (include/piso.h):
  * cells of a block are numbered i + nx*(j + ny*k) (x fastest); blocks are
    concatenated in block order; fields are SoA [component][N];
  * a block side is 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z;  the tangential axes of a side are
    the two other axes in increasing order (t0 fastest);
  * a side is tiled by one or more segments; a 'connect' segment joins the opposite
    side of another (or the same) block with identical axis orientation;
  * Dirichlet boundary values are one array [d][NB]: Dirichlet segments in the order
    they are listed, faces inside a segment in tangential order (t0 fastest).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

CONNECT = "connect"
DIRICHLET = "dirichlet"


@dataclass
class Side:
    """One segment of one block side (a full side is a single segment)."""
    block: int
    side: int
    kind: str
    begin: Tuple[int, int] = (0, 0)
    end: Optional[Tuple[int, int]] = None      # exclusive; None = to the end of the side
    other_block: int = -1                      # connect: block on the other side
    other_begin: Tuple[int, int] = (0, 0)      # connect: tangential start on the other side


@dataclass
class Domain:
    dim: int
    blocks: List[Tuple[int, int, int]]          # (nx, ny, nz); nz = 1 in 2D
    sides: List[Side]
    T: np.ndarray                               # [d, d, N], T[j, i, P] = d xi^j / d x_i
    J: np.ndarray                               # [N], det(d x / d xi) > 0
    centres: Optional[np.ndarray] = None        # [d, N] physical cell centres (diagnostics only)
    # optional metrics on the Dirichlet faces, in u_b's face order (None: those of the
    # boundary cell): Tb[j, i, f] = d xi^j / d x_i and Jb[f] at the face
    Tb: Optional[np.ndarray] = None             # [d, d, NB]
    Jb: Optional[np.ndarray] = None             # [NB]

    @property
    def n_cells(self) -> int:
        return int(sum(nx * ny * nz for nx, ny, nz in self.blocks))

    def block_offsets(self) -> List[int]:
        off = [0]
        for nx, ny, nz in self.blocks:
            off.append(off[-1] + nx * ny * nz)
        return off


def side_tangential_extent(block: Tuple[int, int, int], side: int, dim: int) -> Tuple[int, int]:
    """Extent of the two tangential axes of a block side (second is 1 in 2D)."""
    n = list(block[:dim])
    axis = side // 2
    others = [n[a] for a in range(dim) if a != axis]
    while len(others) < 2:
        others.append(1)
    return others[0], others[1]


def segment_extent(dom: Domain, s: Side) -> Tuple[Tuple[int, int], Tuple[int, int]]:
    t0n, t1n = side_tangential_extent(dom.blocks[s.block], s.side, dom.dim)
    end = s.end if s.end is not None else (t0n, t1n)
    return tuple(s.begin), tuple(end)


def dirichlet_segments(dom: Domain):
    """[(side index, face offset in u_b, n faces)] for the Dirichlet segments, in order."""
    out, off = [], 0
    for si, s in enumerate(dom.sides):
        if s.kind != DIRICHLET:
            continue
        (b0, b1), (e0, e1) = segment_extent(dom, s)
        n = (e0 - b0) * (e1 - b1)
        out.append((si, off, n))
        off += n
    return out


def n_boundary_faces(dom: Domain) -> int:
    segs = dirichlet_segments(dom)
    return segs[-1][1] + segs[-1][2] if segs else 0


def boundary_values(dom: Domain, per_side_value) -> np.ndarray:
    """Fill u_b [d, NB]; per_side_value(side_index) -> constant vector of length d."""
    nb = n_boundary_faces(dom)
    ub = np.zeros((dom.dim, nb))
    for si, off, n in dirichlet_segments(dom):
        ub[:, off:off + n] = np.asarray(per_side_value(si), dtype=np.float64)[:, None]
    return ub


# --------------------------------------------------------------------------- meshes

def tanh_vertices(n: int, beta: float, lo: float, hi: float) -> np.ndarray:
    """n+1 vertices on [lo, hi] clustered towards both ends with a tanh map."""
    s = np.linspace(-1.0, 1.0, n + 1)
    x = np.tanh(beta * s) / math.tanh(beta)
    return lo + (hi - lo) * 0.5 * (x + 1.0)


def tensor_metrics(vertices: List[np.ndarray]):
    """Diagonal metrics of a tensor-product grid from its 1D vertex arrays.

    Returns T [d,d,N], J [N], centres [d,N] in block cell order (x fastest).
    """
    d = len(vertices)
    widths = [np.diff(v) for v in vertices]
    mids = [0.5 * (v[1:] + v[:-1]) for v in vertices]
    grids_w = np.meshgrid(*widths[::-1], indexing="ij")[::-1]   # each [nz,ny,nx] or [ny,nx]
    grids_c = np.meshgrid(*mids[::-1], indexing="ij")[::-1]
    n = grids_w[0].size
    T = np.zeros((d, d, n))
    J = np.ones(n)
    centres = np.zeros((d, n))
    for a in range(d):
        w = grids_w[a].reshape(-1)
        T[a, a] = 1.0 / w
        J *= w
        centres[a] = grids_c[a].reshape(-1)
    return T, J, centres


def vertex_metrics(X: np.ndarray):
    """Cell-centre metrics from structured vertex coordinates.

    X has shape [d, nx+1, ny+1] (2D) or [d, nx+1, ny+1, nz+1] (3D), indexed [coord, i, j(, k)].
    d x / d xi^a at a cell centre is the mean of the cell's edges along axis a (exact
    for affine cells).  Returns T [d,d,N], J [N], centres [d,N] with x fastest.
    """
    d = X.shape[0]
    if d == 2:
        ex = 0.5 * ((X[:, 1:, :-1] - X[:, :-1, :-1]) + (X[:, 1:, 1:] - X[:, :-1, 1:]))
        ey = 0.5 * ((X[:, :-1, 1:] - X[:, :-1, :-1]) + (X[:, 1:, 1:] - X[:, 1:, :-1]))
        edges = [ex, ey]
        c = 0.25 * (X[:, :-1, :-1] + X[:, 1:, :-1] + X[:, :-1, 1:] + X[:, 1:, 1:])
    else:
        def avg4(A):
            return 0.25 * A
        ex = (X[:, 1:, :-1, :-1] - X[:, :-1, :-1, :-1]) + (X[:, 1:, 1:, :-1] - X[:, :-1, 1:, :-1]) \
            + (X[:, 1:, :-1, 1:] - X[:, :-1, :-1, 1:]) + (X[:, 1:, 1:, 1:] - X[:, :-1, 1:, 1:])
        ey = (X[:, :-1, 1:, :-1] - X[:, :-1, :-1, :-1]) + (X[:, 1:, 1:, :-1] - X[:, 1:, :-1, :-1]) \
            + (X[:, :-1, 1:, 1:] - X[:, :-1, :-1, 1:]) + (X[:, 1:, 1:, 1:] - X[:, 1:, :-1, 1:])
        ez = (X[:, :-1, :-1, 1:] - X[:, :-1, :-1, :-1]) + (X[:, 1:, :-1, 1:] - X[:, 1:, :-1, :-1]) \
            + (X[:, :-1, 1:, 1:] - X[:, :-1, 1:, :-1]) + (X[:, 1:, 1:, 1:] - X[:, 1:, 1:, :-1])
        edges = [avg4(ex), avg4(ey), avg4(ez)]
        c = 0.125 * sum(X[:, i0:i0 + X.shape[1] - 1, j0:j0 + X.shape[2] - 1, k0:k0 + X.shape[3] - 1]
                        for i0 in (0, 1) for j0 in (0, 1) for k0 in (0, 1))
    # M[i, a] = d x_i / d xi^a, per cell; transpose spatial axes so that x is fastest
    M = np.stack(edges, axis=1)                        # [d(coord), d(axis), nx, ny(, nz)]
    perm = (0, 1) + tuple(range(M.ndim - 1, 1, -1))
    M = np.transpose(M, perm).reshape(d, d, -1)        # cells in (k, j, i) C-order => x fastest
    c = np.transpose(c, (0,) + tuple(range(c.ndim - 1, 0, -1))).reshape(d, -1)
    Mc = np.moveaxis(M, 2, 0)                          # [N, d, d]
    J = np.linalg.det(Mc)
    Tc = np.linalg.inv(Mc)                             # [N, a, i] = d xi^a / d x_i
    T = np.moveaxis(Tc, 0, 2).copy()                   # [a, i, N]
    return T, J, c


def concat_blocks(parts):
    T = np.concatenate([p[0] for p in parts], axis=2)
    J = np.concatenate([p[1] for p in parts])
    c = np.concatenate([p[2] for p in parts], axis=1)
    return T, J, c


def periodic_sides(block: int, dim: int, axes) -> List[Side]:
    out = []
    for a in axes:
        out.append(Side(block, 2 * a, CONNECT, other_block=block))
        out.append(Side(block, 2 * a + 1, CONNECT, other_block=block))
    return out


# --------------------------------------------------------------------------- cases

@dataclass
class Case:
    name: str
    domain: Domain
    u0: np.ndarray                 # [d, N]
    p0: np.ndarray                 # [N]
    S: np.ndarray                  # [d, N]
    nu: float
    dt: float
    u_b: np.ndarray                # [d, NB]
    n_steps: int
    extra: dict = field(default_factory=dict)


def taylor_green(n: int = 32, nu: float = 0.01, dt: float = 0.01, n_steps: int = 20,
                 amplitude: float = 1.0) -> Case:
    """2D Taylor-Green vortex on a periodic [0, 2pi)^2 block (the first configuration)."""
    v = np.linspace(0.0, 2 * math.pi, n + 1)
    T, J, c = tensor_metrics([v, v])
    dom = Domain(2, [(n, n, 1)], periodic_sides(0, 2, (0, 1)), T, J, c)
    x, y = c
    u0 = amplitude * np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)])
    # Euler balance grad p = -(u . grad) u gives p = +(cos 2x + cos 2y)/4 for this field
    p0 = 0.25 * amplitude ** 2 * (np.cos(2 * x) + np.cos(2 * y))
    return Case("tgv%d" % n, dom, u0, p0, np.zeros_like(u0), nu, dt, np.zeros((2, 0)), n_steps)


def lid_cavity(n: int = 256, beta: float = 1.5, nu: float = 1e-3, n_steps: int = 500,
               lid_speed: float = 1.0, cfl: float = 0.8) -> Case:
    """2D lid-driven cavity on [0,1]^2, tanh wall stretching, lid on the top side."""
    v = tanh_vertices(n, beta, 0.0, 1.0)
    T, J, c = tensor_metrics([v, v])
    sides = [Side(0, s, DIRICHLET) for s in range(4)]
    dom = Domain(2, [(n, n, 1)], sides, T, J, c)
    lid = np.array([lid_speed, 0.0])
    ub = boundary_values(dom, lambda si: lid if dom.sides[si].side == 3 else np.zeros(2))
    dt = cfl * float(np.min(np.diff(v))) / lid_speed
    u0 = np.zeros((2, dom.n_cells))
    return Case("cavity%d" % n, dom, u0, np.zeros(dom.n_cells), np.zeros_like(u0), nu, dt, ub,
                n_steps, {"beta": beta})


def channel_modes(seed: int = 3):
    rng = np.random.default_rng(seed)
    kx = np.repeat(np.array([1.0, 2.0, 3.0, 4.0]), 4)
    kz = np.tile(np.array([2.0, 4.0, 6.0, 8.0]), 4)
    a = rng.standard_normal((3, 16))
    phi = rng.uniform(0.0, 2 * math.pi, (3, 16))
    return kx, kz, a, phi


def channel(nx: int = 96, ny: int = 96, nz: int = 96, beta: float = 1.5, re_tau: float = 180.0,
            n_steps: int = 16, seed: int = 3, cfl: float = 0.1, perturbation: float = 0.1) -> Case:
    """3D channel: x in [0,2pi) and z in [0,pi) periodic, tanh-stretched y in [-1,1] with
    no-slip walls, constant streamwise forcing u_tau^2/delta = 1, nu = 1/Re_tau.

    Initial field: laminar profile with centre-line velocity Re_cl*nu, where
    Re_cl = (Re_tau/0.116)^(1/0.88) as in App. B's channel set-up, plus a seeded,
    analytically divergence-free perturbation u' = curl psi that vanishes at the walls.
    """
    xv = np.linspace(0.0, 2 * math.pi, nx + 1)
    yv = tanh_vertices(ny, beta, -1.0, 1.0)
    zv = np.linspace(0.0, math.pi, nz + 1)
    T, J, c = tensor_metrics([xv, yv, zv])
    sides = periodic_sides(0, 3, (0, 2)) + [Side(0, 2, DIRICHLET), Side(0, 3, DIRICHLET)]
    dom = Domain(3, [(nx, ny, nz)], sides, T, J, c)
    nu = 1.0 / re_tau
    re_cl = (re_tau / 0.116) ** (1.0 / 0.88)
    u_cl = re_cl * nu
    x, y, z = c
    kx, kz, a, ph = channel_modes(seed)
    f = (1.0 - y * y) ** 2
    fp = -4.0 * y * (1.0 - y * y)
    # psi_c = f(y) sum_m a_cm cos(kx x + kz z + ph_cm);  u' = curl psi
    dpsi = {}
    for comp in range(3):
        arg = kx[:, None] * x[None] + kz[:, None] * z[None] + ph[comp][:, None]
        cs = np.cos(arg)
        sn = np.sin(arg)
        s_cos = (a[comp][:, None] * cs).sum(0)
        dpsi[(comp, 'x')] = -f * (a[comp][:, None] * kx[:, None] * sn).sum(0)
        dpsi[(comp, 'y')] = fp * s_cos
        dpsi[(comp, 'z')] = -f * (a[comp][:, None] * kz[:, None] * sn).sum(0)
    up = np.stack([dpsi[(2, 'y')] - dpsi[(1, 'z')],
                   dpsi[(0, 'z')] - dpsi[(2, 'x')],
                   dpsi[(1, 'x')] - dpsi[(0, 'y')]])
    up *= perturbation * u_cl / np.max(np.abs(up))
    u0 = up.copy()
    u0[0] += u_cl * (1.0 - y * y)
    S = np.zeros_like(u0)
    S[0] = 1.0
    speed = sum(np.abs(T[j, 0] * u0[0] + T[j, 1] * u0[1] + T[j, 2] * u0[2]) for j in range(3))
    dt = cfl / float(np.max(speed))
    ub = boundary_values(dom, lambda si: np.zeros(3))
    return Case("channel%dx%dx%d" % (nx, ny, nz), dom, u0, np.zeros(dom.n_cells), S, nu, dt, ub,
                n_steps, {"u_cl": u_cl, "beta": beta, "y": y})


def channel_loss_targets(case: Case, seed: int = 4):
    """Seeded target profiles for the channel statistics loss: u_hat(y), uv_hat(y)."""
    nx, ny, nz = case.domain.blocks[0]
    u0 = case.u0.reshape(3, nz, ny, nx)
    ubar0 = u0[0].mean(axis=(0, 2))
    y = case.extra["y"].reshape(nz, ny, nx)[0, :, 0]
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(ny)
    xi2 = rng.standard_normal(ny)
    u_hat = ubar0 * (1.0 + 0.05 * xi)
    uv_hat = 0.05 * case.extra["u_cl"] ** 2 * (1.0 - y * y) * xi2
    return u_hat, uv_hat


def poiseuille(nx: int = 4, ny: int = 8, nu: float = 1.0, G: float = 1.0, dt: float = 1e6,
               vertices_y: Optional[np.ndarray] = None) -> Case:
    """Plane Poiseuille flow: periodic x, no-slip walls at y = 0 and y = 1, forcing G."""
    xv = np.linspace(0.0, 1.0, nx + 1)
    yv = np.linspace(0.0, 1.0, ny + 1) if vertices_y is None else vertices_y
    T, J, c = tensor_metrics([xv, yv])
    sides = periodic_sides(0, 2, (0,)) + [Side(0, 2, DIRICHLET), Side(0, 3, DIRICHLET)]
    dom = Domain(2, [(nx, len(yv) - 1, 1)], sides, T, J, c)
    S = np.zeros((2, dom.n_cells))
    S[0] = G
    ub = boundary_values(dom, lambda si: np.zeros(2))
    return Case("poiseuille", dom, np.zeros((2, dom.n_cells)), np.zeros(dom.n_cells), S, nu, dt,
                ub, 4)


def sheared_periodic(n: int = 16, shear: float = 1.0, length: float = 2 * math.pi) -> Domain:
    """Affine, non-orthogonal periodic 2D grid: x = xi*h + shear*eta*h, y = eta*h."""
    h = length / n
    xi, eta = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    X = np.stack([xi * h + shear * eta * h, eta * h]).astype(np.float64)
    T, J, c = vertex_metrics(X)
    return Domain(2, [(n, n, 1)], periodic_sides(0, 2, (0, 1)), T, J, c)


def sheared_channel(nx: int = 6, ny: int = 8, shear: float = 0.5, nu: float = 1.0, G: float = 1.0,
                    dt: float = 1e6) -> Case:
    """Poiseuille flow on a skewed periodic grid x = xi*hx + shear*y, walls at y = 0, 1."""
    hx, hy = 1.0 / nx, 1.0 / ny
    xi, eta = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    X = np.stack([xi * hx + shear * eta * hy, eta * hy]).astype(np.float64)
    T, J, c = vertex_metrics(X)
    sides = periodic_sides(0, 2, (0,)) + [Side(0, 2, DIRICHLET), Side(0, 3, DIRICHLET)]
    dom = Domain(2, [(nx, ny, 1)], sides, T, J, c)
    S = np.zeros((2, dom.n_cells))
    S[0] = G
    ub = boundary_values(dom, lambda si: np.zeros(2))
    return Case("sheared_channel", dom, np.zeros((2, dom.n_cells)), np.zeros(dom.n_cells), S, nu,
                dt, ub, 4)


def cylinder_oh(n_theta: int = 256, n_r: int = 128, n_out: int = 128, r_in: float = 0.5,
                r_mid: float = 2.0, half_box: float = 8.0, nu: float = 0.01,
                n_steps: int = 64, cfl: float = 0.8, u_max: float = 1.5) -> Case:
    """2D flow past a cylinder on a conformal 5-block O-H grid.

    Block 0 is the annulus r in [r_in, r_mid] with axes (xi0 = r outward, xi1 = theta
    counter-clockwise, periodic).  Its outer side is split into four segments of
    n_theta/4 faces, each joined to a transition block k = 1..4 that blends a quarter
    arc (centred on +x, +y, -x, -y) into one side of the square [-half_box, half_box]^2.
    Transition blocks have axes (xi0 outward, xi1 counter-clockwise) and join each
    other along the diagonals.  The square sides carry u = (1, 0), the cylinder wall
    u = 0.  All connections keep the axis orientation.
    """
    q = n_theta // 4
    th0 = -math.pi / 4
    # annulus
    r = np.linspace(r_in, r_mid, n_r + 1)
    th = th0 + 2 * math.pi * np.arange(n_theta + 1) / n_theta
    R, TH = np.meshgrid(r, th, indexing="ij")
    X0 = np.stack([R * np.cos(TH), R * np.sin(TH)])
    parts = [vertex_metrics(X0)]
    blocks = [(n_r, n_theta, 1)]
    # transition blocks
    corners = [(half_box, -half_box), (half_box, half_box), (-half_box, half_box),
               (-half_box, -half_box), (half_box, -half_box)]
    for k in range(4):
        s = np.arange(q + 1) / q
        ang = th0 + k * math.pi / 2 + s * math.pi / 2
        inner = np.stack([r_mid * np.cos(ang), r_mid * np.sin(ang)])           # [2, q+1]
        c0, c1 = np.array(corners[k]), np.array(corners[k + 1])
        outer = c0[:, None] + (c1 - c0)[:, None] * s[None]
        t = np.arange(n_out + 1) / n_out
        X = inner[:, None, :] * (1 - t)[None, :, None] + outer[:, None, :] * t[None, :, None]
        parts.append(vertex_metrics(X))
        blocks.append((n_out, q, 1))
    T, J, c = concat_blocks(parts)
    sides = [Side(0, 0, DIRICHLET), Side(0, 2, CONNECT, other_block=0),
             Side(0, 3, CONNECT, other_block=0)]
    for k in range(4):
        sides.append(Side(0, 1, CONNECT, begin=(k * q, 0), end=((k + 1) * q, 1),
                          other_block=1 + k, other_begin=(0, 0)))
    for k in range(4):
        b = 1 + k
        sides.append(Side(b, 0, CONNECT, other_block=0, other_begin=(k * q, 0)))
        sides.append(Side(b, 1, DIRICHLET))
        sides.append(Side(b, 2, CONNECT, other_block=1 + (k - 1) % 4))
        sides.append(Side(b, 3, CONNECT, other_block=1 + (k + 1) % 4))
    dom = Domain(2, blocks, sides, T, J, c)
    inflow = np.array([1.0, 0.0])
    ub = boundary_values(dom, lambda si: np.zeros(2) if dom.sides[si].block == 0 else inflow)
    u0 = np.zeros((2, dom.n_cells))
    u0[0] = 1.0
    speed = sum(np.sqrt(T[j, 0] ** 2 + T[j, 1] ** 2) for j in range(2))
    dt = cfl / float(np.max(u_max * speed))
    return Case("cylinder5", dom, u0, np.zeros(dom.n_cells), np.zeros_like(u0), nu, dt, ub,
                n_steps)


def segment_mask(dom: Domain, pick) -> np.ndarray:
    """Boolean mask over the Dirichlet faces [NB]: True on the faces of every Dirichlet
    segment whose index si in dom.sides satisfies pick(si)."""
    mask = np.zeros(n_boundary_faces(dom), dtype=bool)
    for si, off, n in dirichlet_segments(dom):
        if pick(si):
            mask[off:off + n] = True
    return mask


def open_channel(nx: int = 32, ny: int = 16, length: float = 4.0, u_in: float = 1.0,
                 nu: float = 0.01, cfl: float = 0.5, beta: float = 1.2, n_steps: int = 16) -> Case:
    """2D channel [0, length] x [0, 1]: parabolic inflow u = 4 u_in y (1 - y) on the
    -x side, an advective outflow on the +x side (extra["outflow"], the face mask, and
    extra["u_m"], the characteristic velocity), no-slip walls at y = 0, 1 with
    tanh-clustered rows."""
    xv = np.linspace(0.0, length, nx + 1)
    yv = tanh_vertices(ny, beta, 0.0, 1.0)
    T, J, c = tensor_metrics([xv, yv])
    sides = [Side(0, 0, DIRICHLET), Side(0, 1, DIRICHLET), Side(0, 2, DIRICHLET), Side(0, 3, DIRICHLET)]
    dom = Domain(2, [(nx, ny, 1)], sides, T, J, c)
    yc = 0.5 * (yv[1:] + yv[:-1])
    prof = 4.0 * u_in * yc * (1.0 - yc)
    ub = np.zeros((2, n_boundary_faces(dom)))
    for si, off, n in dirichlet_segments(dom):
        if si in (0, 1):                 # -x inflow and +x outflow (initial value)
            ub[0, off:off + n] = prof
    u0 = np.zeros((2, dom.n_cells))
    u0[0] = prof.repeat(nx)
    outflow = segment_mask(dom, lambda si: si == 1)
    dt = cfl * float(np.min(np.diff(xv))) / u_in
    return Case("open_channel", dom, u0, np.zeros(dom.n_cells), np.zeros_like(u0), nu, dt, ub,
                n_steps, extra={"outflow": outflow, "u_m": np.array([u_in, 0.0])})


def random_fields(case: Case, seed: int, scale: float = 1.0):
    """Seeded random velocity/pressure/source/boundary perturbations of a case (tests)."""
    rng = np.random.default_rng(seed)
    d, n = case.u0.shape
    return (scale * rng.standard_normal((d, n)), scale * rng.standard_normal(n),
            scale * rng.standard_normal((d, n)), scale * rng.standard_normal(case.u_b.shape))
