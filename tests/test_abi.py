"""C-ABI library checks that need no GPU: the built library loads and exports every
function include/piso.h declares, the binding covers the same set, and the host-side
division magic used by the kernels' cell indexing is exact."""
import ctypes
import os
import random
import subprocess

import pytest

from paper_2505_16992_amd import _lib as L


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = L.declared_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(L._SIGS) == set(names)


def test_library_exports_nothing_else():
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines() if " T piso_" in ln})
    assert exported == L.declared_symbols()


def test_default_opts_without_device():
    lib = L.load()
    o = L.StepOpts()
    lib.piso_default_step_opts(L.PISO_MIXED, ctypes.byref(o))
    assert o.n_correctors == 2 and o.grad_p_in_predictor == 1
    assert o.pres.rtol == pytest.approx(1e-8)
    lib.piso_default_step_opts(L.PISO_F64, ctypes.byref(o))
    assert o.pres.rtol == pytest.approx(1e-10) and o.vel.rtol == pytest.approx(1e-10)
    assert o.report_flux_div == 0


def test_step_opts_layout_matches_library():
    """piso_default_step_opts clears sizeof(piso_step_opts) bytes: in a buffer with a canary
    after the binding's structure, the canary survives (the binding is not shorter than the
    library's struct) and the last field is cleared (not longer)."""
    lib = L.load()
    n = ctypes.sizeof(L.StepOpts)
    buf = (ctypes.c_uint8 * (n + 64))(*([0xAB] * (n + 64)))
    lib.piso_default_step_opts(L.PISO_F32, ctypes.cast(buf, ctypes.POINTER(L.StepOpts)))
    assert all(b == 0xAB for b in buf[n:])
    o = L.StepOpts.from_buffer(buf)
    assert o.report_flux_div == 0 and o.adjoint_warm_start == 1 and o.n_correctors == 2
    assert o.p_prev is None and o.p_prev_star is None and o.p_star_out is None and o.u_prev is None


def _magic(d):
    l = 0
    while (1 << l) < d:
        l += 1
    return ((1 << (31 + l)) + d - 1) // d, 31 + l


@pytest.mark.parametrize("d", [1, 2, 3, 5, 7, 96, 127, 128, 192, 255, 256, 1000, 9216, 24576, 65535, 36864])
def test_division_magic_exact(d):
    m, s = _magic(d)
    rng = random.Random(d)
    samples = [0, 1, d - 1, d, d + 1, (1 << 31) - 1] + [rng.randrange(0, 1 << 31) for _ in range(2000)]
    for n in samples:
        assert (n * m) >> s == n // d
    assert m * ((1 << 31) - 1) < (1 << 64)


def _header_structs():
    """Field names of every 'typedef struct { ... } name;' in include/piso.h, in order
    (comments removed; several declarators per line split; array sizes dropped)."""
    import os
    import re
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "piso.h")
    text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct \{(.*?)\}\s*(\w+);", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            first, *rest = decl.split(",")
            names = [first.split()[-1]] + [r.strip() for r in rest]
            fields += [re.sub(r"\[.*\]", "", n).lstrip("*") for n in names]
        out[name] = fields
    return out


@pytest.mark.parametrize("c_name, py", [("piso_side_desc", "SideDesc"), ("piso_domain_desc", "DomainDesc"),
                                        ("piso_solve_opts", "SolveOpts"), ("piso_solve_info", "SolveInfo"),
                                        ("piso_step_opts", "StepOpts"), ("piso_step_info", "StepInfo"),
                                        ("piso_system", "System"), ("piso_system_grad", "SystemGrad")])
def test_binding_structs_follow_the_header(c_name, py):
    """The ctypes structures list the header's fields in the header's order."""
    fields = _header_structs()[c_name]
    assert [f[0] for f in getattr(L, py)._fields_] == fields
