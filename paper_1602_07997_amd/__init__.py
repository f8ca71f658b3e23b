"""MI355X-native nodal discontinuous Galerkin wave step (acoustic / elastic).

The hot path lives in ``libdgwave.so`` (HIP for gfx950, C ABI declared in
``include/dgwave.h``); this package only marshals arguments to it.  The
library is loaded on first use of any of the names below, so that the build
module can run before it exists.
"""

__all__ = ["DGBatch", "DGMisfit", "DGSolver", "misfit", "mesh_connectivity", "ref_sizes", "reference_operators"]


def __getattr__(name):
    if name in ("DGMisfit", "misfit"):
        from . import adjoint

        return getattr(adjoint, name)
    if name in __all__:
        from . import solver

        return getattr(solver, name)
    raise AttributeError(name)
