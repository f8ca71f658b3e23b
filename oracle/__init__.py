"""FP64 CPU oracle of the nodal discontinuous Galerkin wave solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU hot path computes: the reference
tetrahedron (nodes, differentiation, mass and lift matrices), the affine
geometry and face connectivity of a tetrahedral mesh, the acoustic and
isotropic elastic right-hand sides with upwind fluxes (Sec. 2.1 and 2.2 of
the paper, eqs. (2)-(6) and the unnumbered elastic right-hand side), the
third-order Adams-Bashforth update (eq. (4)) and the discrete energy.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  The product library never calls it, and it
shares no code with the product: the only module both use is ``dginputs``
(seeded synthetic meshes, coefficient fields and initial-data functions),
which holds none of the method's arithmetic.
"""

from .refelem import RefElement, reference_element  # noqa: F401
from .mesh import MeshGeometry, build_mesh  # noqa: F401
from .dg import (  # noqa: F401
    AcousticOracle,
    ElasticOracle,
    ab3_coefficients,
    make_oracle,
)
