"""MI355X (gfx950) proximal-gradient solver for the CONCORD / PseudoNet estimator.

The iteration runs in hand-written HIP kernels behind the C-ABI of
``include/concord.h`` (libconcord.so); ``_lib`` is the ctypes binding and
``autograd`` the differentiable smooth objective.
"""
from ._lib import (  # noqa: F401
    Solver, Batch, TorchAllocator, ConcordError, StepInfo, SolveInfo, load, EXPORTED, LIB_PATH,
    concord_version, concord_suggest_variant,
)

__all__ = ["Solver", "Batch", "ConcordError", "StepInfo", "SolveInfo", "load"]
