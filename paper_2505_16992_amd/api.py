"""Python API over the PISO C-ABI: contexts, one step, its adjoint, an autograd
Function and a checkpointed rollout.

PyTorch supplies device memory and the stream; every computation is done by the HIP
kernels behind libpiso.so.  Tensors are SoA: a vector field is [d, N], a scalar [N],
Dirichlet values [d, NB], viscosity [1] (global) or [N] (per cell).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_KIND = {"connect": L.PISO_SIDE_CONNECT, "dirichlet": L.PISO_SIDE_DIRICHLET}
_PREC = {"f64": L.PISO_F64, "f32": L.PISO_F32, "mixed": L.PISO_MIXED}


class PisoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("piso error %d: %s" % (code, msg))
        self.code = code


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _tangential(block, side, dim):
    axis = side // 2
    others = [block[a] for a in range(dim) if a != axis]
    while len(others) < 2:
        others.append(1)
    return others


class Context:
    """A block layout, its metrics and the solver workspaces on the current device.

    domain: any object with .dim, .blocks [(nx, ny, nz)], .sides (objects with block,
    side, kind in {'connect', 'dirichlet'}, begin, end (None = whole side), other_block,
    other_begin), .T [d, d, N] and .J [N] (numpy float64).
    """

    def __init__(self, domain, precision: str = "f32"):
        self.lib = L.lib()
        self.precision = precision
        self.prec = _PREC[precision]
        self.dim = int(domain.dim)
        self.dtype = torch.float32 if self.prec == L.PISO_F32 else torch.float64   # MIXED stores double
        cells = np.array([list(b) for b in domain.blocks], dtype=np.int32).reshape(-1)
        sides = (L.SideDesc * len(domain.sides))()
        for q, s in enumerate(domain.sides):
            t0n, t1n = _tangential(domain.blocks[s.block], s.side, self.dim)
            end = s.end if s.end is not None else (t0n, t1n)
            sides[q].block, sides[q].side, sides[q].kind = s.block, s.side, _KIND[s.kind]
            sides[q].begin[0], sides[q].begin[1] = s.begin
            sides[q].end[0], sides[q].end[1] = end
            sides[q].other_block = s.other_block
            sides[q].other_begin[0], sides[q].other_begin[1] = s.other_begin
        T = np.ascontiguousarray(domain.T, dtype=np.float64)
        J = np.ascontiguousarray(domain.J, dtype=np.float64)
        # metrics on the Dirichlet faces (u_b's face order), or None: the boundary cells'
        Tb, Jb = getattr(domain, "Tb", None), getattr(domain, "Jb", None)
        dptr = C.POINTER(C.c_double)
        if Tb is not None:
            Tb = np.ascontiguousarray(Tb, dtype=np.float64)
            Jb = np.ascontiguousarray(Jb, dtype=np.float64)
            nb = sum((sd.end[0] - sd.begin[0]) * (sd.end[1] - sd.begin[1])
                     for sd in sides if sd.kind == L.PISO_SIDE_DIRICHLET)
            if Tb.shape != (self.dim, self.dim, nb) or Jb.shape != (nb,):
                raise ValueError("face metrics: Tb [d, d, %d] and Jb [%d] expected" % (nb, nb))
        self._keep = (cells, sides, T, J, Tb, Jb)
        desc = L.DomainDesc(self.dim, len(domain.blocks), len(domain.sides),
                            cells.ctypes.data_as(C.POINTER(C.c_int32)), sides,
                            T.ctypes.data_as(dptr), J.ctypes.data_as(dptr),
                            None if Tb is None else Tb.ctypes.data_as(dptr),
                            None if Jb is None else Jb.ctypes.data_as(dptr))
        h = C.c_void_p()
        rc = self.lib.piso_create(C.byref(desc), self.prec, C.byref(h))
        if rc != 0:
            raise PisoError(rc, self.lib.piso_create_error().decode())
        self.h = h
        self._adj_owner = None   # the rollout (or step) whose backward wrote the warm-start history
        self.device = torch.device("cuda", torch.cuda.current_device())
        n, nb, tb, eb = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        no = C.c_int32()
        self.lib.piso_sizes(h, C.byref(n), C.byref(nb), C.byref(tb), C.byref(eb), C.byref(no))
        self.N, self.NB, self.tape_bytes, self.elem_bytes = n.value, nb.value, tb.value, eb.value
        self.non_orthogonal = bool(no.value)
        nl = C.c_int32()
        cells_l, slots_l = (C.c_int64 * 16)(), (C.c_int32 * 16)()
        self.lib.piso_mg_info(h, C.byref(nl), cells_l, slots_l)
        self.mg_levels = [(int(cells_l[q]), int(slots_l[q])) for q in range(nl.value)]
        la = C.c_int32(0)
        self._check(self.lib.piso_mg_smoother(self.h, C.byref(la)), "piso_mg_smoother")
        self.mg_line_axis = int(la.value)   # 0: point Jacobi on the fine level, 1/2: lines along y/z
        zg = C.c_int32(0)
        self._check(self.lib.piso_mg_marching(self.h, C.byref(zg)), "piso_mg_marching")
        self.mg_marching_groups = int(zg.value)   # > 0: the plane-marching fine-grid kernels run

    def __del__(self):
        h = getattr(self, "h", None)
        try:
            if h is not None and h.value:
                self.lib.piso_destroy(h)
                self.h = None
        except Exception:      # interpreter shutdown: the library may already be gone
            pass

    # ---------------------------------------------------------------- helpers
    def _check(self, rc, what):
        if rc < 0:
            raise PisoError(rc, "%s: %s" % (what, self.lib.piso_last_error(self.h).decode()))
        return rc

    def _t(self, x, shape, name, allow_none=False):
        if x is None:
            if allow_none:
                return None
            raise ValueError("%s is required" % name)
        if x.device != self.device or x.dtype != self.dtype:
            raise ValueError("%s must be a %s tensor on %s" % (name, self.dtype, self.device))
        if tuple(x.shape) != tuple(shape):
            raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(x.shape)))
        if not x.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        return x

    def _nu(self, nu):
        if nu.numel() == 1:
            return self._t(nu.reshape(1), (1,), "nu"), 0
        return self._t(nu, (self.N,), "nu"), 1

    def _ub(self, u_b):
        if self.NB == 0:
            return None
        return self._t(u_b, (self.dim, self.NB), "u_b")

    def zeros(self, *shape):
        return torch.zeros(*shape, dtype=self.dtype, device=self.device)

    def default_opts(self) -> L.StepOpts:
        o = L.StepOpts()
        self.lib.piso_default_step_opts(self.prec, C.byref(o))
        return o

    def new_tape(self):
        return torch.empty(self.tape_bytes // self.elem_bytes, dtype=self.dtype, device=self.device)

    def new_system(self):
        d, N = self.dim, self.N
        z = self.zeros
        return {"A": z(N), "C": z(2, d, N), "b_u": z(d, N), "b": z(d, N), "Pf": z(d, N),
                "Dinv": z(N), "h": z(d, N), "rhs": z(N)}

    @staticmethod
    def _sys(t):
        return L.System(*[t[k].data_ptr() for k in ("A", "C", "b_u", "b", "Pf", "Dinv", "h", "rhs")])

    def new_system_grad(self):
        d, N = self.dim, self.N
        z = self.zeros
        return {"dA": z(N), "dC": z(2, d, N), "db_u": z(d, N), "db": z(d, N)}

    @staticmethod
    def _gsys(g):
        return L.SystemGrad(*[g[k].data_ptr() for k in ("dA", "dC", "db_u", "db")])

    # ---------------------------------------------------------------- whole step
    def step(self, u, p, nu, S, u_b, dt, opts=None, tape=None, info=False, p_prev=None, p_prev_star=None,
             p_star_out=None, u_prev=None):
        """One PISO step.  Optional starts of its linear solves from the previous step of
        the same rollout: u_prev and p_prev, that step's input velocity and pressure, and
        p_prev_star, its first-corrector pressure p* (which p_star_out, if given, receives
        for this step); see piso_step_opts."""
        d, N = self.dim, self.N
        self._t(u, (d, N), "u")
        self._t(p, (N,), "p")
        for x, nm in ((p_prev, "p_prev"), (p_prev_star, "p_prev_star"), (p_star_out, "p_star_out")):
            if x is not None:
                self._t(x, (N,), nm)
        if u_prev is not None:
            self._t(u_prev, (d, N), "u_prev")
        self._t(S, (d, N), "S")
        nu_t, nf = self._nu(nu)
        ub = self._ub(u_b)
        if tape is not None:
            self._t(tape, (self.tape_bytes // self.elem_bytes,), "tape")
        o = opts if opts is not None else self.default_opts()
        if any(x is not None for x in (p_prev, p_prev_star, p_star_out, u_prev)):
            o = L.StepOpts.from_buffer_copy(o)
            o.p_prev = _ptr(p_prev)
            o.p_prev_star = _ptr(p_prev_star)
            o.p_star_out = _ptr(p_star_out)
            o.u_prev = _ptr(u_prev)
        u1 = torch.empty_like(u)
        p1 = torch.empty_like(p)
        inf = L.StepInfo()
        rc = self.lib.piso_step(self.h, _stream(), _ptr(u), _ptr(p), _ptr(nu_t), nf, _ptr(S), _ptr(ub),
                                float(dt), _ptr(u1), _ptr(p1), _ptr(tape), C.byref(o), C.byref(inf))
        self._check(rc, "piso_step")
        return (u1, p1, inf.as_dict()) if info else (u1, p1)

    def step_backward(self, tape, u, p, nu, u_b, dt, du1, dp1, opts=None, want=("u", "p", "S", "nu", "u_b"),
                      info=False):
        d, N = self.dim, self.N
        nu_t, nf = self._nu(nu)
        ub = self._ub(u_b)
        o = opts if opts is not None else self.default_opts()
        du = self.zeros(d, N) if "u" in want else None
        dp = self.zeros(N) if "p" in want else None
        dS = self.zeros(d, N) if "S" in want else None
        dnu = self.zeros(nu_t.shape[0]) if "nu" in want else None
        dub = self.zeros(d, self.NB) if ("u_b" in want and self.NB) else None
        du1 = None if du1 is None else self._t(du1.contiguous(), (d, N), "du1")
        dp1 = None if dp1 is None else self._t(dp1.contiguous(), (N,), "dp1")
        inf = L.StepInfo()
        rc = self.lib.piso_step_backward(self.h, _stream(), _ptr(tape), _ptr(u), _ptr(p), _ptr(nu_t), nf,
                                         _ptr(ub), float(dt), _ptr(du1), _ptr(dp1), _ptr(du), _ptr(dp),
                                         _ptr(dS), _ptr(dnu), _ptr(dub), C.byref(o), C.byref(inf))
        self._check(rc, "piso_step_backward")
        out = {"u": du, "p": dp, "S": dS, "nu": dnu, "u_b": dub}
        return (out, inf.as_dict()) if info else out

    def adjoint_reset(self):
        """Start the next step_backward's adjoint pressure solves from zero (see
        adjoint_warm_start in the step options)."""
        self._adj_owner = None
        return self._check(self.lib.piso_adjoint_reset(self.h), "piso_adjoint_reset")

    # ---------------------------------------------------------------- fine-grained calls
    def assemble(self, sys, u, p, nu, S, u_b, dt, grad_p_in_predictor=1):
        nu_t, nf = self._nu(nu)
        rc = self.lib.piso_assemble(self.h, _stream(), _ptr(u), _ptr(p), _ptr(nu_t), nf, _ptr(S),
                                    _ptr(self._ub(u_b)), float(dt), int(grad_p_in_predictor),
                                    C.byref(self._sys(sys)))
        return self._check(rc, "piso_assemble")

    def solve_velocity(self, sys, u_star, opts: L.SolveOpts):
        inf = L.SolveInfo()
        rc = self.lib.piso_solve_velocity(self.h, _stream(), C.byref(self._sys(sys)), _ptr(u_star),
                                          C.byref(opts), C.byref(inf))
        self._check(rc, "piso_solve_velocity")
        return inf.as_dict()

    def solve_velocity_noalloc(self, sys, u_star, opts: L.SolveOpts):
        """solve_velocity with its workspace in the library's fixed per-GPU array (no
        allocation during the call; calls on one GPU must not overlap)."""
        inf = L.SolveInfo()
        rc = self.lib.piso_solve_velocity_noalloc(self.h, _stream(), C.byref(self._sys(sys)), _ptr(u_star),
                                                  C.byref(opts), C.byref(inf))
        self._check(rc, "piso_solve_velocity_noalloc")
        return inf.as_dict()

    def solve_pressure(self, sys, u_in, u_b, p_lag, p, opts: L.SolveOpts):
        inf = L.SolveInfo()
        rc = self.lib.piso_solve_pressure(self.h, _stream(), C.byref(self._sys(sys)), _ptr(u_in),
                                          _ptr(self._ub(u_b)), _ptr(p_lag), _ptr(p), C.byref(opts),
                                          C.byref(inf))
        self._check(rc, "piso_solve_pressure")
        return inf.as_dict()

    def correct(self, sys, p, p_lag, u_b, u_out, F_out=None):
        rc = self.lib.piso_correct(self.h, _stream(), C.byref(self._sys(sys)), _ptr(p), _ptr(p_lag),
                                   _ptr(self._ub(u_b)), _ptr(u_out), _ptr(F_out))
        return self._check(rc, "piso_correct")

    def correct_backward(self, sys, p, du_out, dh, dp, dA):
        rc = self.lib.piso_correct_backward(self.h, _stream(), C.byref(self._sys(sys)), _ptr(p),
                                            _ptr(du_out), _ptr(dh), _ptr(dp), _ptr(dA))
        return self._check(rc, "piso_correct_backward")

    def solve_pressure_backward(self, sys, u_in, p_lag, p, dh, dp, du_in, dp_lag, du_b, g, opts,
                                skip_solve=False):
        inf = L.SolveInfo()
        rc = self.lib.piso_solve_pressure_backward(
            self.h, _stream(), C.byref(self._sys(sys)), _ptr(u_in), _ptr(p_lag), _ptr(p), _ptr(dh), _ptr(dp),
            _ptr(du_in), _ptr(dp_lag), _ptr(du_b), C.byref(self._gsys(g)), int(skip_solve), C.byref(opts),
            C.byref(inf))
        self._check(rc, "piso_solve_pressure_backward")
        return inf.as_dict()

    def solve_velocity_backward(self, sys, u_star, du_star, g, opts, skip_solve=False):
        inf = L.SolveInfo()
        rc = self.lib.piso_solve_velocity_backward(self.h, _stream(), C.byref(self._sys(sys)), _ptr(u_star),
                                                   _ptr(du_star), C.byref(self._gsys(g)), int(skip_solve),
                                                   C.byref(opts), C.byref(inf))
        self._check(rc, "piso_solve_velocity_backward")
        return inf.as_dict()

    def assemble_backward(self, u_n, nu, u_b, dt, g, du_n, dp_n, dS, dnu, du_b, grad_p_in_predictor=1):
        nu_t, nf = self._nu(nu)
        rc = self.lib.piso_assemble_backward(self.h, _stream(), _ptr(u_n), _ptr(nu_t), nf, _ptr(self._ub(u_b)),
                                             float(dt), int(grad_p_in_predictor), C.byref(self._gsys(g)),
                                             _ptr(du_n), _ptr(dp_n), _ptr(dS), _ptr(dnu), _ptr(du_b))
        return self._check(rc, "piso_assemble_backward")

    # ---------------------------------------------------------------- diagnostics
    def outflow_mask(self, mask):
        """Device int32 [NB] outflow flags from a boolean/integer array."""
        m = torch.as_tensor(np.asarray(mask).astype(np.int32), device=self.device)
        if tuple(m.shape) != (self.NB,):
            raise ValueError("outflow mask must have shape (%d,)" % self.NB)
        return m.contiguous()

    def _mask(self, mask):
        if mask.device != self.device or mask.dtype != torch.int32 or tuple(mask.shape) != (self.NB,):
            raise ValueError("outflow mask must be an int32 tensor of shape (%d,) on %s" % (self.NB, self.device))
        return mask.contiguous()

    def outflow_update(self, u, u_b, mask, u_m, dt, out=None):
        """Advective outflow update of the Dirichlet values before a step."""
        d, N = self.dim, self.N
        self._t(u, (d, N), "u")
        ub = self._t(u_b, (d, self.NB), "u_b")
        m = self._mask(mask)
        um = (C.c_double * 3)(*[float(x) for x in list(u_m)[:d]])
        out = torch.empty_like(ub) if out is None else self._t(out, (d, self.NB), "out")
        self._check(self.lib.piso_outflow_update(self.h, _stream(), _ptr(u), _ptr(ub), _ptr(m), um, float(dt),
                                                 _ptr(out)), "piso_outflow_update")
        return out

    def outflow_update_backward(self, u, u_b, mask, u_m, dt, dub_out, du=None):
        """(du_b, du) for the gradient dub_out of the updated values; du (if given) is
        accumulated into, else a new tensor is returned."""
        d, N = self.dim, self.N
        m = self._mask(mask)
        um = (C.c_double * 3)(*[float(x) for x in list(u_m)[:d]])
        g = self._t(dub_out.contiguous(), (d, self.NB), "dub_out")
        dub = torch.empty_like(g)
        du = self.zeros(d, N) if du is None else self._t(du, (d, N), "du")
        self._check(self.lib.piso_outflow_update_backward(self.h, _stream(), _ptr(u), _ptr(u_b), _ptr(m), um,
                                                          float(dt), _ptr(g), _ptr(du), _ptr(dub)),
                    "piso_outflow_update_backward")
        return dub, du

    def divfree_gradient(self, S, dS, lam, opts=None, info=False):
        """(dS + lam grad p_S, p_S) with P(A = 1) p_S = div S (eq. SgradPsgrad)."""
        d, N = self.dim, self.N
        self._t(S, (d, N), "S")
        g = self._t(dS.contiguous(), (d, N), "dS")
        o = opts if opts is not None else self.default_opts().pres
        out = torch.empty_like(g)
        p = self.zeros(N)
        inf = L.SolveInfo()
        self._check(self.lib.piso_divfree_gradient(self.h, _stream(), _ptr(S), _ptr(g), float(lam), C.byref(o),
                                                   _ptr(out), _ptr(p), C.byref(inf)), "piso_divfree_gradient")
        return (out, p, inf.as_dict()) if info else (out, p)

    # ---------------------------------------------------------------- statistics
    def stats_size(self, axis=1):
        n, r = C.c_int64(), C.c_int64()
        self._check(self.lib.piso_stats_size(self.h, int(axis), C.byref(n), C.byref(r)), "piso_stats_size")
        return n.value, r.value

    def stats_state(self, axis=1):
        """Empty statistics state (device float64)."""
        n, r = self.stats_size(axis)
        return torch.zeros(n, r, dtype=torch.float64, device=self.device)

    def stats_accumulate(self, u, state, axis=1):
        self._t(u, (self.dim, self.N), "u")
        self._check(self.lib.piso_stats_accumulate(self.h, _stream(), _ptr(u), int(axis), _ptr(state)),
                    "piso_stats_accumulate")
        return state

    def stats_finalize(self, state, axis=1):
        n, _ = self.stats_size(axis)
        npair = self.dim * (self.dim + 1) // 2
        mean = torch.empty(n, self.dim, dtype=torch.float64, device=self.device)
        cov = torch.empty(n, npair, dtype=torch.float64, device=self.device)
        self._check(self.lib.piso_stats_finalize(self.h, _stream(), int(axis), _ptr(state), _ptr(mean), _ptr(cov)),
                    "piso_stats_finalize")
        return mean, cov

    def stats_backward(self, u, state, mean_bar, cov_bar, axis=1, du=None):
        du = self.zeros(self.dim, self.N) if du is None else self._t(du, (self.dim, self.N), "du")
        mb = mean_bar.to(torch.float64).contiguous()
        cb = cov_bar.to(torch.float64).contiguous()
        self._check(self.lib.piso_stats_backward(self.h, _stream(), _ptr(u), int(axis), _ptr(state), _ptr(mb),
                                                 _ptr(cb), _ptr(du)), "piso_stats_backward")
        return du

    # ------------------------------------------------ arbitrary-order moments, budget terms
    def moments_size(self, m, order, axis=1):
        n, r = C.c_int64(), C.c_int64()
        self._check(self.lib.piso_moments_size(self.h, int(axis), int(m), int(order), C.byref(n), C.byref(r)),
                    "piso_moments_size")
        return n.value, r.value

    def moments_state(self, m, order, axis=1):
        """Empty state of the order-`order` comoments of m variables (device float64)."""
        n, r = self.moments_size(m, order, axis)
        return torch.zeros(n, r, dtype=torch.float64, device=self.device)

    def moments_accumulate(self, x, state, order, axis=1):
        m = x.shape[0]
        self._t(x, (m, self.N), "x")
        self._check(self.lib.piso_moments_accumulate(self.h, _stream(), _ptr(x), int(m), int(order), int(axis),
                                                     _ptr(state)), "piso_moments_accumulate")
        return state

    def moments_finalize(self, state, m, order, axis=1):
        """(mean [n_planes, m], central moments [n_planes, n_alpha]) in the storage order
        of the multi-indices (by order, then lexicographic tuples)."""
        n, r = self.moments_size(m, order, axis)
        mean = torch.empty(n, m, dtype=torch.float64, device=self.device)
        mom = torch.empty(n, r - 1 - m, dtype=torch.float64, device=self.device)
        self._check(self.lib.piso_moments_finalize(self.h, _stream(), int(m), int(order), int(axis), _ptr(state),
                                                   _ptr(mean), _ptr(mom)), "piso_moments_finalize")
        return mean, mom

    def moments_backward(self, x, state, mean_bar, mom_bar, order, axis=1, dx=None):
        m = x.shape[0]
        dx = self.zeros(m, self.N) if dx is None else self._t(dx, (m, self.N), "dx")
        mb = mean_bar.to(torch.float64).contiguous()
        ob = mom_bar.to(torch.float64).contiguous()
        self._check(self.lib.piso_moments_backward(self.h, _stream(), _ptr(x), int(m), int(order), int(axis),
                                                   _ptr(state), _ptr(mb), _ptr(ob), _ptr(dx)), "piso_moments_backward")
        return dx

    def field_gradient(self, phi, phi_b=None):
        """[d, ncomp, N] cell-centred gradient of phi [ncomp, N] (ghost 2 phi_b - phi_P across
        Dirichlet faces, or phi_P when phi_b is None)."""
        nc = phi.shape[0]
        self._t(phi, (nc, self.N), "phi")
        if phi_b is not None:
            self._t(phi_b, (nc, self.NB), "phi_b")
        out = torch.empty(self.dim, nc, self.N, dtype=self.dtype, device=self.device)
        self._check(self.lib.piso_field_gradient(self.h, _stream(), _ptr(phi), int(nc), _ptr(phi_b), _ptr(out)),
                    "piso_field_gradient")
        return out

    def budget(self, state_u, state_grad, state_up, order_u, wall_mean, axis=1):
        """Budget terms {P, eps, T, D, Pi: [n_planes, d(d+1)/2]} from accumulated states."""
        n, _ = self.moments_size(self.dim, order_u, axis)
        npair = self.dim * (self.dim + 1) // 2
        out = torch.empty(5, n, npair, dtype=torch.float64, device=self.device)
        wm = (C.c_double * (2 * self.dim))(*[float(v) for v in np.asarray(wall_mean, dtype=np.float64).ravel()])
        self._check(self.lib.piso_budget(self.h, _stream(), int(axis), int(order_u), _ptr(state_u),
                                         _ptr(state_grad.contiguous()), _ptr(state_up), wm, _ptr(out)),
                    "piso_budget")
        return dict(zip(("P", "eps", "T", "D", "Pi"), out))

    def set_timing(self, enable: bool):
        self.lib.piso_set_timing(self.h, int(enable))

    def get_timing(self):
        """{kernel class: (total ms, launches)} since timing was enabled."""
        out = {}
        for k, name in enumerate(L.TIME_KINDS):
            ms, n = C.c_double(), C.c_int64()
            self._check(self.lib.piso_get_timing(self.h, k, C.byref(ms), C.byref(n)), "piso_get_timing")
            out[name] = (ms.value, n.value)
        return out


# ===================================================================== autograd

def _adjoint_owner(pctx: Context, owner):
    """Before a backward step: the context's adjoint warm-start history (the adjoint
    pressure solutions of its last backward step) is kept only for the backward pass
    that wrote it.  Every rollout, and every stand-alone step, is its own owner; the
    first backward step of another owner clears the history, so gradients depend on
    the rollout (or step) alone, whatever was differentiated before and whichever of
    its states the loss uses."""
    if pctx._adj_owner is not owner:
        pctx.adjoint_reset()
        pctx._adj_owner = owner


def _chained_step(pctx: Context, u, p, nu, S, u_b, dt, opts, start, tape=None):
    """One step whose linear solves start from the previous step of the rollout
    (start = (u_prev, p_prev, p_prev_star) or None; see piso_step_opts).  Returns
    (u^{n+1}, p^{n+1}, p*): p* is this step's first-corrector pressure, the next step's
    p_prev_star, so the next step's start is (u, p, p*)."""
    uv, pv, pvs = start if start is not None else (None, None, None)
    pst = torch.empty_like(p)
    u1, p1 = pctx.step(u, p, nu, S, u_b, dt, opts, tape=tape, p_prev=pv, p_prev_star=pvs, p_star_out=pst,
                       u_prev=uv)
    return u1, p1, pst


class PisoStep(torch.autograd.Function):
    """One differentiable PISO step: (u, p, S, nu, u_b) -> (u^{n+1}, p^{n+1}), plus the
    step's first-corrector pressure p* (not differentiable) for the next step's start.

    The forward keeps a tape of the intermediates; the backward runs the hand-written
    adjoint (transposed solves and per-operation adjoints).  `owner` groups the steps
    of one rollout for the adjoint warm start (None: a stand-alone step).  u_prev,
    p_prev and p_prev_star only choose where the linear solves start (piso_step_opts)."""

    @staticmethod
    def forward(fctx, pctx: Context, opts, dt, owner, u, p, S, nu, u_b, u_prev=None, p_prev=None, p_prev_star=None):
        tape = pctx.new_tape()
        start = _segment_start(u_prev, p_prev, p_prev_star)
        u1, p1, pst = _chained_step(pctx, u, p, nu, S, u_b, dt, opts, start, tape=tape)
        fctx.pctx, fctx.opts, fctx.dt = pctx, opts, dt
        fctx.owner = owner if owner is not None else object()
        fctx.save_for_backward(tape, u, p, nu, u_b if u_b is not None else torch.empty(0))
        fctx.has_ub = u_b is not None
        fctx.mark_non_differentiable(pst)
        return u1, p1, pst

    @staticmethod
    def backward(fctx, du1, dp1, _dpst):
        tape, u, p, nu, u_b = fctx.saved_tensors
        pctx = fctx.pctx
        _adjoint_owner(pctx, fctx.owner)
        g = pctx.step_backward(tape, u, p, nu, u_b if fctx.has_ub else None, fctx.dt, du1, dp1, fctx.opts)
        return (None, None, None, None, g["u"], g["p"], g["S"], g["nu"].reshape(nu.shape),
                g["u_b"] if fctx.has_ub else None, None, None, None)


def _segment_start(u_prev, p_prev, p_prev_star):
    if u_prev is None and p_prev is None and p_prev_star is None:
        return None
    return tuple(None if x is None else x.detach() for x in (u_prev, p_prev, p_prev_star))


class _Segment(torch.autograd.Function):
    """k steps whose tapes are dropped in the forward and recomputed in the backward
    (step checkpointing): memory O(1 state + k tapes) per segment.  The pressure starts
    chain through the segment (chain = True) from (p_prev, p_prev_star), in the forward
    and in its recomputation alike; the last step's start pair for the next step is
    returned beside the state (not differentiable)."""

    @staticmethod
    def forward(fctx, pctx: Context, opts, dt, k, owner, chain, u, p, S, nu, u_b, u_prev, p_prev, p_prev_star):
        start = _segment_start(u_prev, p_prev, p_prev_star)
        fctx.start = start
        uu, pp = u, p
        for _ in range(k):
            lu, lp = uu, pp
            uu, pp, pst = _chained_step(pctx, uu, pp, nu, S, u_b, dt, opts, start)
            start = (lu, lp, pst) if chain else None
        fctx.pctx, fctx.opts, fctx.dt, fctx.k, fctx.owner = pctx, opts, dt, k, owner
        fctx.chain = chain
        fctx.has_ub = u_b is not None
        fctx.save_for_backward(u, p, S, nu, u_b if u_b is not None else torch.empty(0))
        nxt = (lu.detach().clone(), lp.detach().clone(), pst)
        fctx.mark_non_differentiable(*nxt)
        return (uu, pp) + nxt

    @staticmethod
    def backward(fctx, du, dp, _d1, _d2, _d3):
        u, p, S, nu, u_b = fctx.saved_tensors
        pctx, opts, dt, k = fctx.pctx, fctx.opts, fctx.dt, fctx.k
        ub = u_b if fctx.has_ub else None
        states, tapes = [(u, p)], []
        uu, pp, start = u, p, fctx.start
        for _ in range(k):
            t = pctx.new_tape()
            lu, lp = uu, pp
            uu, pp, pst = _chained_step(pctx, uu, pp, nu, S, ub, dt, opts, start, tape=t)
            start = (lu, lp, pst) if fctx.chain else None
            states.append((uu, pp))
            tapes.append(t)
        dS = torch.zeros_like(S)
        dnu = torch.zeros_like(nu.reshape(-1))
        dub = torch.zeros_like(ub) if ub is not None else None
        gu, gp = du, dp
        _adjoint_owner(pctx, fctx.owner)
        for q in range(k - 1, -1, -1):
            un, pn = states[q]
            g = pctx.step_backward(tapes[q], un, pn, nu, ub, dt, gu, gp, opts)
            gu, gp = g["u"], g["p"]
            dS += g["S"]
            dnu += g["nu"]
            if dub is not None:
                dub += g["u_b"]
            tapes[q] = None
        return None, None, None, None, None, None, gu, gp, dS, dnu.reshape(nu.shape), dub, None, None, None


class OutflowUpdate(torch.autograd.Function):
    """Differentiable advective outflow update (u, u_b) -> u_b' applied before a step."""

    @staticmethod
    def forward(fctx, pctx: Context, mask, u_m, dt, u, u_b):
        fctx.pctx, fctx.mask, fctx.u_m, fctx.dt = pctx, mask, u_m, dt
        fctx.save_for_backward(u, u_b)
        return pctx.outflow_update(u, u_b, mask, u_m, dt)

    @staticmethod
    def backward(fctx, dub_out):
        u, u_b = fctx.saved_tensors
        dub, du = fctx.pctx.outflow_update_backward(u, u_b, fctx.mask, fctx.u_m, fctx.dt, dub_out)
        return None, None, None, None, du, dub


class _OutflowSegment(torch.autograd.Function):
    """k checkpointed steps, each preceded by the outflow update of the boundary
    values: (u, p, S, nu, u_b) -> (u^{n+k}, p^{n+k}, u_b^{n+k}), with the pressure
    starts chained as in _Segment."""

    @staticmethod
    def forward(fctx, pctx: Context, opts, dt, k, owner, chain, mask, u_m, u, p, S, nu, u_b, u_prev, p_prev,
                p_prev_star):
        start = _segment_start(u_prev, p_prev, p_prev_star)
        fctx.start = start
        uu, pp, bb = u, p, u_b
        for _ in range(k):
            bb = pctx.outflow_update(uu, bb, mask, u_m, dt)
            lu, lp = uu, pp
            uu, pp, pst = _chained_step(pctx, uu, pp, nu, S, bb, dt, opts, start)
            start = (lu, lp, pst) if chain else None
        fctx.pctx, fctx.opts, fctx.dt, fctx.k, fctx.mask, fctx.u_m = pctx, opts, dt, k, mask, u_m
        fctx.owner, fctx.chain = owner, chain
        fctx.save_for_backward(u, p, S, nu, u_b)
        nxt = (lu.detach().clone(), lp.detach().clone(), pst)
        fctx.mark_non_differentiable(*nxt)
        return (uu, pp, bb) + nxt

    @staticmethod
    def backward(fctx, du, dp, dbb, _d1, _d2, _d3):
        u, p, S, nu, u_b = fctx.saved_tensors
        pctx, opts, dt, k, mask, u_m = fctx.pctx, fctx.opts, fctx.dt, fctx.k, fctx.mask, fctx.u_m
        states, tapes, used = [(u, p, u_b)], [], []
        uu, pp, bb, start = u, p, u_b, fctx.start
        for _ in range(k):
            nb = pctx.outflow_update(uu, bb, mask, u_m, dt)
            t = pctx.new_tape()
            lu, lp = uu, pp
            uu, pp, pst = _chained_step(pctx, uu, pp, nu, S, nb, dt, opts, start, tape=t)
            start = (lu, lp, pst) if fctx.chain else None
            used.append(nb)
            states.append((uu, pp, nb))
            tapes.append(t)
            bb = nb
        dS = torch.zeros_like(S)
        dnu = torch.zeros_like(nu.reshape(-1))
        gu, gp = du, dp
        gb = dbb.contiguous() if dbb is not None else torch.zeros_like(u_b)
        _adjoint_owner(pctx, fctx.owner)
        for q in range(k - 1, -1, -1):
            un, pn, bprev = states[q]
            g = pctx.step_backward(tapes[q], un, pn, nu, used[q], dt, gu, gp, opts)
            dS += g["S"]
            dnu += g["nu"]
            gb_used = g["u_b"] + gb
            gb, gu = pctx.outflow_update_backward(un, bprev, mask, u_m, dt, gb_used, du=g["u"])
            gp = g["p"]
            tapes[q] = None
        return None, None, None, None, None, None, None, None, gu, gp, dS, dnu.reshape(nu.shape), gb, None, None, None


class PlaneStatistics(torch.autograd.Function):
    """Mean [n_planes, d] and covariance [n_planes, d(d+1)/2] of fields accumulated over
    homogeneous planes (online merging in the library), differentiable with respect to
    every field."""

    @staticmethod
    def forward(fctx, pctx: Context, axis, *us):
        state = pctx.stats_state(axis)
        for u in us:
            pctx.stats_accumulate(u, state, axis)
        mean, cov = pctx.stats_finalize(state, axis)
        fctx.pctx, fctx.axis = pctx, axis
        fctx.save_for_backward(state, *us)
        return mean, cov

    @staticmethod
    def backward(fctx, mbar, cbar):
        state, *us = fctx.saved_tensors
        pctx = fctx.pctx
        mbar = torch.zeros_like(state[:, 1:1 + pctx.dim]) if mbar is None else mbar
        npair = pctx.dim * (pctx.dim + 1) // 2
        cbar = torch.zeros(state.shape[0], npair, dtype=torch.float64, device=state.device) if cbar is None else cbar
        grads = [pctx.stats_backward(u, state, mbar, cbar, fctx.axis) for u in us]
        return (None, None, *grads)


class PlaneMoments(torch.autograd.Function):
    """Mean [n_planes, m] and central comoments of orders 2..order [n_planes, n_alpha] of
    fields x [m, N] accumulated over homogeneous planes, differentiable with respect to
    every field."""

    @staticmethod
    def forward(fctx, pctx: Context, order, axis, *xs):
        m = xs[0].shape[0]
        state = pctx.moments_state(m, order, axis)
        for x in xs:
            pctx.moments_accumulate(x, state, order, axis)
        mean, mom = pctx.moments_finalize(state, m, order, axis)
        fctx.pctx, fctx.order, fctx.axis = pctx, order, axis
        fctx.save_for_backward(state, *xs)
        return mean, mom

    @staticmethod
    def backward(fctx, mbar, obar):
        state, *xs = fctx.saved_tensors
        pctx, m = fctx.pctx, xs[0].shape[0]
        na = state.shape[1] - 1 - m
        mbar = torch.zeros(state.shape[0], m, dtype=torch.float64, device=state.device) if mbar is None else mbar
        obar = torch.zeros(state.shape[0], na, dtype=torch.float64, device=state.device) if obar is None else obar
        grads = [pctx.moments_backward(x, state, mbar, obar, fctx.order, fctx.axis) for x in xs]
        return (None, None, None, *grads)


def plane_moments(pctx: Context, xs, order, axis=1):
    """(mean, moments) of orders 2..order over the fields `xs` (list of [m, N] tensors)."""
    return PlaneMoments.apply(pctx, order, axis, *xs)


class TurbulenceBudget:
    """Online statistics for the turbulent energy budget of Sec. 2.5 over the planes
    normal to `axis` of a single-block context: per accumulated step the velocity's
    moments up to `order` (>= 3), the covariances of its gradients du/dx_k and the
    covariance of (u, grad p); `terms(wall_mean)` evaluates P, eps, T, D and Pi."""

    def __init__(self, pctx: Context, axis=1, order=4):
        d = pctx.dim
        self.pctx, self.axis, self.order = pctx, axis, order
        self.su = pctx.moments_state(d, order, axis)
        self.sg = torch.stack([pctx.moments_state(d, 2, axis) for _ in range(d)])
        self.sup = pctx.moments_state(2 * d, 2, axis)

    def accumulate(self, u, p, u_b=None):
        c = self.pctx
        c.moments_accumulate(u, self.su, self.order, self.axis)
        g = c.field_gradient(u, u_b)
        for k in range(c.dim):
            c.moments_accumulate(g[k].contiguous(), self.sg[k], 2, self.axis)
        gp = c.field_gradient(p.reshape(1, -1), None)[:, 0]
        c.moments_accumulate(torch.cat([u, gp]).contiguous(), self.sup, 2, self.axis)

    def moments(self):
        return self.pctx.moments_finalize(self.su, self.pctx.dim, self.order, self.axis)

    def terms(self, wall_mean):
        return self.pctx.budget(self.su, self.sg, self.sup, self.order, wall_mean, self.axis)


def plane_statistics(pctx: Context, us, axis=1):
    """(mean, cov) over the fields `us` (list of [d, N] tensors)."""
    return PlaneStatistics.apply(pctx, axis, *us)


class DivFreeGradient(torch.autograd.Function):
    """Identity on a learned source S whose backward adds lam grad p_S to the incoming
    gradient (eq. SgradPsgrad)."""

    @staticmethod
    def forward(fctx, pctx: Context, lam, opts, S):
        fctx.pctx, fctx.lam, fctx.opts = pctx, lam, opts
        fctx.save_for_backward(S)
        return S.clone()

    @staticmethod
    def backward(fctx, gS):
        (S,) = fctx.saved_tensors
        g, _ = fctx.pctx.divfree_gradient(S.detach(), gS, fctx.lam, fctx.opts)
        return None, None, None, g


def divfree_gradient_hook(pctx: Context, S, lam, opts=None):
    """S unchanged in the forward; its gradient gains lam grad p_S in the backward."""
    return DivFreeGradient.apply(pctx, lam, opts, S)


def step(pctx: Context, u, p, S, nu, u_b, dt, opts=None):
    """Differentiable single step (keeps its tape until backward)."""
    u1, p1, _ = PisoStep.apply(pctx, opts if opts is not None else pctx.default_opts(), dt, None, u, p, S, nu, u_b)
    return u1, p1


def rollout(pctx: Context, u0, p0, S, nu, u_b, dt, n_steps: int, checkpoint_every: int = 0, opts=None,
            warmup: int = 0, return_all: bool = False, outflow=None, extrapolate: bool = True):
    """n_steps differentiable steps.  checkpoint_every = 0 keeps every tape; k > 0
    stores only the state at the start of each k-step segment and recomputes the
    segment's tapes in the backward.  warmup steps run first without a tape.

    return_all: the list of states after every step (k = 0), or after every segment
    (k > 0: the states inside a segment are not kept, only its last one).  The adjoint
    pressure solves of the rollout's backward warm-start from each other but never
    from another rollout's (or step's) backward.

    outflow = (mask, u_m): before every step the Dirichlet values of the masked faces
    are advanced by the advective outflow update (the boundary values then become part
    of the state; the result gains a third entry, the final u_b).

    extrapolate: every step after the first starts its linear solves from the previous
    step's fields (piso_step_opts.u_prev, p_prev and p_prev_star: the velocity solve from
    2 u_n - u_{n-1}, corrector 1 from p*_{n-1} + (p_n - p_{n-1}), corrector 2 from
    p* + (p_n - p*_{n-1})); the chain runs through warm-up steps and checkpointed
    segments alike, so that results do not depend on checkpoint_every."""
    o = opts if opts is not None else pctx.default_opts()
    owner = object()   # the backward steps of this rollout share the adjoint warm start
    u, p, ub = u0, p0, u_b
    start = None   # (u_{n-1}, p_{n-1}, p*_{n-1}) of the previous step, once there is one
    if outflow is not None:
        mask, u_m = outflow
        mask = pctx._mask(mask)
    if warmup:
        with torch.no_grad():
            ub = None if ub is None else ub.detach()
            for _ in range(warmup):
                if outflow is not None:
                    ub = pctx.outflow_update(u.detach(), ub, mask, u_m, dt)
                lu, lp = u.detach(), p.detach()
                u, p, pst = _chained_step(pctx, lu, lp, nu.detach(), S.detach(), ub, dt, o, start)
                start = (lu, lp, pst) if extrapolate else None
    traj = []
    done = 0
    uv, pv, pvs = start if start is not None else (None, None, None)
    while done < n_steps:
        lu, lp = u.detach(), p.detach()
        if outflow is not None:
            if checkpoint_every > 0:
                k = min(checkpoint_every, n_steps - done)
                u, p, ub, lu, lp, pst = _OutflowSegment.apply(pctx, o, dt, k, owner, extrapolate, mask, u_m, u, p,
                                                              S, nu, ub, uv, pv, pvs)
                done += k
            else:
                ub = OutflowUpdate.apply(pctx, mask, u_m, dt, u, ub)
                u, p, pst = PisoStep.apply(pctx, o, dt, owner, u, p, S, nu, ub, uv, pv, pvs)
                done += 1
        elif checkpoint_every > 0:
            k = min(checkpoint_every, n_steps - done)
            u, p, lu, lp, pst = _Segment.apply(pctx, o, dt, k, owner, extrapolate, u, p, S, nu, ub, uv, pv, pvs)
            done += k
        else:
            u, p, pst = PisoStep.apply(pctx, o, dt, owner, u, p, S, nu, ub, uv, pv, pvs)
            done += 1
        uv, pv, pvs = (lu, lp, pst) if extrapolate else (None, None, None)
        if return_all:
            traj.append((u, p) if outflow is None else (u, p, ub))
    if return_all:
        return traj
    return (u, p) if outflow is None else (u, p, ub)
