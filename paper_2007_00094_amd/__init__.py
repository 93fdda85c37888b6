"""MI355X library for the second-order invariant-domain-preserving Q1 scheme
for the compressible Euler equations (Maier & Kronbichler, arXiv:2007.00094).

The per-stage edge sweep (graph viscosity, low-order update and bounds,
high-order directions, convex limiting in two passes, SSP-RK3) runs in HIP
kernels for gfx950 behind the C-ABI of include/idp.h; ``capi`` binds it and
``Solver`` wraps it for torch device tensors.  ``inputs`` holds the seeded
synthetic meshes and initial states.
"""
from . import inputs  # noqa: F401


def Solver(*args, **kwargs):
    """Construct a solver (imports torch and loads libidp.so on first use)."""
    from .solver import Solver as _S
    return _S(*args, **kwargs)
