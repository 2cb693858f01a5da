"""Multi-block adjacency for the oracle (Sec. 2.2 and App. A.4 of the paper).

Each block is a regular grid; each block side is tiled by segments that either connect
to another block with matching resolution (a conformal connection; a block joined to
itself gives periodicity) or prescribe a Dirichlet velocity.  For every cell P and
every face (axis j, side s) the oracle records either the neighbour cell F (>= 0) or
-1 - b for the b-th Dirichlet boundary face.

Parity: pinned by the brute-force dense tests, which build their own neighbour lookup
with plain loops, and by the topology validation tests.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from cases import CONNECT, DIRICHLET, Domain, segment_extent, side_tangential_extent


class TopologyError(ValueError):
    pass


@dataclass
class Topology:
    dim: int
    n_cells: int
    nbr: np.ndarray          # [N, d, 2] int64: neighbour index or -1 - boundary face
    n_bfaces: int
    bface_cell: np.ndarray   # [NB] cell owning each Dirichlet face
    bface_axis: np.ndarray   # [NB]
    bface_side: np.ndarray   # [NB] 0 = low side, 1 = high side


def _cell_index(off, nx, ny, i, j, k):
    return off + i + nx * (j + ny * k)


def _tangential(axis, i, j, k):
    if axis == 0:
        return j, k
    if axis == 1:
        return i, k
    return i, j


def _from_tangential(axis, along, t0, t1):
    if axis == 0:
        return along, t0, t1
    if axis == 1:
        return t0, along, t1
    return t0, t1, along


def build_topology(dom: Domain) -> Topology:
    d = dom.dim
    off = dom.block_offsets()
    N = off[-1]
    UNSET = np.iinfo(np.int64).min
    nbr = np.full((N, d, 2), UNSET, dtype=np.int64)

    # interior neighbours
    for b, (nx, ny, nz) in enumerate(dom.blocks):
        n = (nx, ny, nz)
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        idx = _cell_index(off[b], nx, ny, i, j, k)
        pos = (i, j, k)
        for a in range(d):
            stride = (1, nx, nx * ny)[a]
            lo = pos[a] > 0
            hi = pos[a] < n[a] - 1
            nbr[idx[lo], a, 0] = idx[lo] - stride
            nbr[idx[hi], a, 1] = idx[hi] + stride

    # boundary faces from the side segments
    bcell, baxis, bside = [], [], []
    nbf = 0
    for seg in dom.sides:
        if not (0 <= seg.block < len(dom.blocks)) or not (0 <= seg.side < 2 * d):
            raise TopologyError("bad block/side in segment %r" % (seg,))
        nx, ny, nz = dom.blocks[seg.block]
        n = (nx, ny, nz)
        a, s = seg.side // 2, seg.side % 2
        (b0, b1), (e0, e1) = segment_extent(dom, seg)
        t0n, t1n = side_tangential_extent(dom.blocks[seg.block], seg.side, d)
        if not (0 <= b0 < e0 <= t0n and 0 <= b1 < e1 <= t1n):
            raise TopologyError("segment out of range: %r" % (seg,))
        along = 0 if s == 0 else n[a] - 1
        for t1 in range(b1, e1):
            for t0 in range(b0, e0):
                i, j, k = _from_tangential(a, along, t0, t1)
                P = _cell_index(off[seg.block], nx, ny, i, j, k)
                if nbr[P, a, s] != UNSET:
                    raise TopologyError("face covered twice: block %d side %d t=(%d,%d)"
                                        % (seg.block, seg.side, t0, t1))
                if seg.kind == DIRICHLET:
                    nbr[P, a, s] = -1 - nbf
                    bcell.append(P)
                    baxis.append(a)
                    bside.append(s)
                    nbf += 1
                elif seg.kind == CONNECT:
                    ob = seg.other_block
                    if not (0 <= ob < len(dom.blocks)):
                        raise TopologyError("bad other block in %r" % (seg,))
                    onx, ony, onz = dom.blocks[ob]
                    on = (onx, ony, onz)
                    o0 = t0 - b0 + seg.other_begin[0]
                    o1 = t1 - b1 + seg.other_begin[1]
                    ot0n, ot1n = side_tangential_extent(dom.blocks[ob], 2 * a + (1 - s), d)
                    if not (0 <= o0 < ot0n and 0 <= o1 < ot1n):
                        raise TopologyError("connection leaves the other block: %r" % (seg,))
                    oalong = 0 if s == 1 else on[a] - 1
                    oi, oj, ok = _from_tangential(a, oalong, o0, o1)
                    nbr[P, a, s] = _cell_index(off[ob], onx, ony, oi, oj, ok)
                else:
                    raise TopologyError("unsupported side kind %r" % (seg.kind,))
    if np.any(nbr == UNSET):
        bad = np.argwhere(nbr == UNSET)[0]
        raise TopologyError("face not covered by any segment: cell %d axis %d side %d" % tuple(bad))
    # conformity: a connection must be reciprocal
    for a in range(d):
        for s in range(2):
            F = nbr[:, a, s]
            m = F >= 0
            back = nbr[F[m], a, 1 - s]
            if not np.array_equal(back, np.nonzero(m)[0]):
                raise TopologyError("non-reciprocal connection along axis %d" % a)
    if np.any(dom.J <= 0):
        raise TopologyError("non-positive Jacobian")
    return Topology(d, N, nbr, nbf, np.array(bcell, dtype=np.int64),
                    np.array(baxis, dtype=np.int64), np.array(bside, dtype=np.int64))
