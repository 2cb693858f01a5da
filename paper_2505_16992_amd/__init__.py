"""MI355X-native differentiable multi-block PISO step (arXiv 2505.16992, PICT).

The compute path is libpiso.so (hand-written HIP for gfx950) behind the C-ABI in
include/piso.h; this package is its thin Python binding.
"""
from ._lib import lib, declared_symbols, LIB_PATH  # noqa: F401


def __getattr__(name):
    # the torch-based API is imported lazily so that the ABI can be inspected without it
    if name in ("Context", "PisoStep", "step", "rollout", "PisoError"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
