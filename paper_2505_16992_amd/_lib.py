"""ctypes binding of libpiso.so (include/piso.h): argument marshalling only.

The library is built in-tree by paper_2505_16992_amd/build.py; importing this module
fails loudly if it is missing.  Every compute call runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpiso.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "piso.h")

PISO_F64, PISO_F32, PISO_MIXED = 0, 1, 2
PISO_OK, PISO_NOT_CONVERGED, PISO_BREAKDOWN = 0, 1, 2
PISO_E_ARG, PISO_E_TOPOLOGY, PISO_E_HIP, PISO_E_NAN, PISO_E_OOM = -1, -2, -3, -4, -5
PISO_SIDE_CONNECT, PISO_SIDE_DIRICHLET = 0, 1
PISO_PRECOND_JACOBI, PISO_PRECOND_MG, PISO_PRECOND_ILU0, PISO_PRECOND_JACOBI_ILU0 = 0, 1, 2, 3
TIME_KINDS = ("cg_stencil", "cg_update", "mg_down0", "mg_up0", "mg_coarse", "cg_update_restrict",
              "mg_smooth0")


class SideDesc(C.Structure):
    _fields_ = [("block", C.c_int32), ("side", C.c_int32), ("kind", C.c_int32),
                ("begin", C.c_int32 * 2), ("end", C.c_int32 * 2), ("other_block", C.c_int32),
                ("other_begin", C.c_int32 * 2)]


class DomainDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_blocks", C.c_int32), ("n_sides", C.c_int32),
                ("block_cells", C.POINTER(C.c_int32)), ("sides", C.POINTER(SideDesc)),
                ("T", C.POINTER(C.c_double)), ("J", C.POINTER(C.c_double)),
                ("Tb", C.POINTER(C.c_double)), ("Jb", C.POINTER(C.c_double))]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("check_every", C.c_int32),
                ("inner_rtol", C.c_double), ("max_refine", C.c_int32), ("precond", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("refinements", C.c_int32),
                ("fallback", C.c_int32), ("rel_residual", C.c_double)]

    def as_dict(self):
        return {"status": self.status, "iters": self.iters, "refinements": self.refinements,
                "fallback": self.fallback, "rel_residual": self.rel_residual}


class StepOpts(C.Structure):
    _fields_ = [("vel", SolveOpts), ("pres", SolveOpts), ("n_correctors", C.c_int32),
                ("grad_p_in_predictor", C.c_int32), ("grad_path_flags", C.c_int32),
                ("adjoint_warm_start", C.c_int32), ("report_flux_div", C.c_int32),
                ("p_prev", C.c_void_p), ("p_prev_star", C.c_void_p), ("p_star_out", C.c_void_p),
                ("u_prev", C.c_void_p)]


class StepInfo(C.Structure):
    _fields_ = [("vel", SolveInfo), ("pres", SolveInfo * 2), ("flux_div_linf", C.c_double * 2)]

    def as_dict(self):
        return {"vel": self.vel.as_dict(), "pres": [self.pres[0].as_dict(), self.pres[1].as_dict()],
                "flux_div_linf": [self.flux_div_linf[0], self.flux_div_linf[1]]}


class System(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("A", "C", "b_u", "b", "Pf", "Dinv", "h", "rhs")]


class SystemGrad(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("dA", "dC", "db_u", "db")]


VP = C.c_void_p
I32 = C.c_int32
F64 = C.c_double

_SIGS = {
    "piso_create": (I32, [C.POINTER(DomainDesc), I32, C.POINTER(VP)]),
    "piso_destroy": (None, [VP]),
    "piso_last_error": (C.c_char_p, [VP]),
    "piso_create_error": (C.c_char_p, []),
    "piso_sizes": (I32, [VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                         C.POINTER(C.c_int64), C.POINTER(I32)]),
    "piso_mg_marching": (I32, [VP, C.POINTER(I32)]),
    "piso_mg_info": (I32, [VP, C.POINTER(I32), C.POINTER(C.c_int64), C.POINTER(I32)]),
    "piso_default_step_opts": (None, [I32, C.POINTER(StepOpts)]),
    "piso_assemble": (I32, [VP, VP, VP, VP, VP, I32, VP, VP, F64, I32, C.POINTER(System)]),
    "piso_solve_velocity": (I32, [VP, VP, C.POINTER(System), VP, C.POINTER(SolveOpts),
                                  C.POINTER(SolveInfo)]),
    "piso_solve_velocity_noalloc": (I32, [VP, VP, C.POINTER(System), VP, C.POINTER(SolveOpts),
                                          C.POINTER(SolveInfo)]),
    "piso_solve_pressure": (I32, [VP, VP, C.POINTER(System), VP, VP, VP, VP, C.POINTER(SolveOpts),
                                  C.POINTER(SolveInfo)]),
    "piso_correct": (I32, [VP, VP, C.POINTER(System), VP, VP, VP, VP, VP]),
    "piso_step": (I32, [VP, VP, VP, VP, VP, I32, VP, VP, F64, VP, VP, VP, C.POINTER(StepOpts),
                        C.POINTER(StepInfo)]),
    "piso_correct_backward": (I32, [VP, VP, C.POINTER(System), VP, VP, VP, VP, VP]),
    "piso_solve_pressure_backward": (I32, [VP, VP, C.POINTER(System), VP, VP, VP, VP, VP, VP, VP,
                                           VP, C.POINTER(SystemGrad), I32, C.POINTER(SolveOpts),
                                           C.POINTER(SolveInfo)]),
    "piso_solve_velocity_backward": (I32, [VP, VP, C.POINTER(System), VP, VP, C.POINTER(SystemGrad),
                                           I32, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "piso_assemble_backward": (I32, [VP, VP, VP, VP, I32, VP, F64, I32, C.POINTER(SystemGrad), VP,
                                     VP, VP, VP, VP]),
    "piso_step_backward": (I32, [VP, VP, VP, VP, VP, VP, I32, VP, F64, VP, VP, VP, VP, VP, VP, VP,
                                 C.POINTER(StepOpts), C.POINTER(StepInfo)]),
    "piso_outflow_update": (I32, [VP, VP, VP, VP, VP, C.POINTER(F64), F64, VP]),
    "piso_outflow_update_backward": (I32, [VP, VP, VP, VP, VP, C.POINTER(F64), F64, VP, VP, VP]),
    "piso_divfree_gradient": (I32, [VP, VP, VP, VP, F64, C.POINTER(SolveOpts), VP, VP, C.POINTER(SolveInfo)]),
    "piso_stats_size": (I32, [VP, I32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "piso_stats_accumulate": (I32, [VP, VP, VP, I32, VP]),
    "piso_stats_finalize": (I32, [VP, VP, I32, VP, VP, VP]),
    "piso_stats_backward": (I32, [VP, VP, VP, I32, VP, VP, VP, VP]),
    "piso_moments_size": (I32, [VP, I32, I32, I32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "piso_moments_accumulate": (I32, [VP, VP, VP, I32, I32, I32, VP]),
    "piso_moments_finalize": (I32, [VP, VP, I32, I32, I32, VP, VP, VP]),
    "piso_moments_backward": (I32, [VP, VP, VP, I32, I32, I32, VP, VP, VP, VP]),
    "piso_field_gradient": (I32, [VP, VP, VP, I32, VP, VP]),
    "piso_budget": (I32, [VP, VP, I32, I32, VP, VP, VP, C.POINTER(C.c_double), VP]),
    "piso_set_timing": (I32, [VP, I32]),
    "piso_adjoint_reset": (I32, [VP]),
    "piso_mg_smoother": (I32, [VP, C.POINTER(I32)]),
    "piso_get_timing": (I32, [VP, I32, C.POINTER(F64), C.POINTER(C.c_int64)]),
}


def declared_symbols():
    """Function names declared in include/piso.h."""
    with open(HEADER) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(piso_[a-z_]+)\s*\(", txt)))


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libpiso.so is not built (run: python -m paper_2505_16992_amd.build)")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib
