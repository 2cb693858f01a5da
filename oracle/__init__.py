"""Plain FP64 CPU oracle of one PISO step and its adjoint (test infrastructure only).

This package is the reference the HIP library is checked against.  It is imported only
by the tests, by the smoke check and by the CPU-baseline leg of the benchmark; the
product path never calls it.  It shares no code with the HIP library: it builds its
own adjacency, assembles explicit SciPy sparse matrices following App. A.2-A.5 of the
paper, and solves them with direct (SuperLU) or FP64 Krylov solves.

All arithmetic is dtype-generic (float64 or complex128) so that complex-step
derivatives can pin the adjoint.

Parity status per function is stated in each module docstring; readings of the paper
where it is silent or ambiguous are listed in the design document and in the
docstrings of the functions that implement them.
"""
from .topology import Topology, build_topology  # noqa: F401
from .piso import Geometry, step, StepRecord  # noqa: F401
from .adjoint import step_vjp  # noqa: F401
