"""MI355X-native pCGMG solver for multi-material SIMP compliance (arXiv 2301.07457).

The compute path is libmtomg.so (HIP, gfx950) behind the C ABI in
include/mtomg.h; ``solver`` wraps it with torch tensors and an autograd
function (``PCGMGSolver`` also exposes the cone filter and the Poisson
model problem of Section 5.1).  Importing this package does not load the library; the first
solver object does, and fails loudly if it is not built.
"""

__all__ = ["PCGMGSolver", "ComplianceFn", "build"]


def __getattr__(name):
    if name in ("PCGMGSolver", "ComplianceFn"):
        from . import solver
        return getattr(solver, name)
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
