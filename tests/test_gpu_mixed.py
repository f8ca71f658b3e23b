"""Mixed-precision MFMA variants (acoustic and elastic) against the FP64 oracle.

The BF16 / FP16 variants split both operands of the volume and LIFT
products into 16-bit halves and accumulate D_hi x_hi + D_hi x_lo + D_lo x_hi
in FP32; fields, r and the update stay FP32.  Bar: relative L2 error
<= 1e-4 against the FP64 oracle, overall and per field, and node by node
1e-3 of each field's largest value, for one right-hand side and for 20 AB3
steps, on 108 elements (several full tiles and a ragged one).
"""

import numpy as np
import pytest
import torch

from oracle.dg import AB3Stepper
from tests._cases import Case, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("variant", ["mfma_bf16", "mfma_f16"])
@pytest.mark.parametrize("N", list(range(1, 9)))
def test_mixed_precision_parity(N, variant, physics):
    log(f"{variant} {physics} N={N}")
    c = Case(physics, N, 0, jitter=0.1, seed=70 + N, coef_kind="random", init="smooth", dims=(3, 2, 3))
    c.solver.variant = variant
    assert c.solver.variant == variant
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    c.check(c.to_host(r), c.oracle.rhs(c.q0), 1e-4, "rhs")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(20, c.dt)
    q = c.to_host(c.solver.get_fields())
    c.check(q, AB3Stepper(c.oracle, c.q0).step(20, c.dt), 1e-4, "20 steps")


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("variant", ["mfma", "mfma_bf16", "mfma_f16"])
def test_mfma_variants_in_batches(variant, physics):
    """A batch of meshes of several degrees on one MFMA variant follows the
    members' own trajectories."""
    from paper_1602_07997_amd import DGBatch, DGSolver

    cases = []
    for i, (N, dims) in enumerate([(2, (2, 3, 2)), (3, (3, 2, 2)), (5, (2, 2, 1)), (3, (2, 2, 2)),
                                   (6, (3, 2, 3))]):
        c = Case(physics, N, None, jitter=0.1, seed=90 + i, coef_kind="random", dims=dims)
        c.solver.variant = variant
        c.solver.set_fields(c.to_gpu(c.q0_gpu))
        t = DGSolver(physics, N, c.mesh.elem_xyz, c.mesh.elem_topo)
        t.set_coefficients(torch.tensor(c.coef, dtype=torch.float32, device="cuda"))
        t.variant = variant
        t.set_fields(c.to_gpu(c.q0_gpu))
        cases.append((c, t))
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    b = DGBatch([c.solver for c, _ in cases], stream=stream, graph=True)
    b.step(14, [c.dt for c, _ in cases])
    for c, t in cases:
        t.step(14, c.dt)
    stream.synchronize()
    torch.cuda.synchronize()
    tol = 1e-5 if variant == "mfma" else 1e-4
    for c, t in cases:
        a_, b_ = c.solver.get_fields().double(), t.get_fields().double()
        assert float(torch.linalg.vector_norm(a_ - b_) / torch.linalg.vector_norm(b_)) <= 1e-6
        c.check(c.to_host(a_), AB3Stepper(c.oracle, c.q0).step(14, c.dt), tol, f"batch member N={c.N} K={c.mesh.K}")
    b.close()
