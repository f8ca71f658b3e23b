"""One right-hand side per (physics, degree, kernel variant) on the ~2M-node
meshes that the benchmark steps, against one FP64 oracle right-hand side.

Meshes and coefficients are those of the benchmark sweeps (Kuhn cube with
n = round((2e6 / (6 Np))^(1/3)) subcubes per edge, jitter 10 % of h, seed 0;
acoustic two-layer (rho, c), elastic log-uniform (rho, lambda, mu), seed 1).
The state is a seeded Gaussian pulse per field (sigma = 0.1, the benchmark's
pulse width), so that every field and its error norm are defined.

Bars.  At these mesh sizes the element size h is 1/44 .. 1/13 while the
pulse varies on a scale of 0.1, so D_j q cancels to a small fraction of
sum_m |D_nm q_m|: that sum exceeds the largest |D q| by about 10^2 (element
size against pulse width, times the N^2 growth of |D|), and every rounding
of a product is amplified by that factor in a node-wise comparison.

* FP32 variants: the 1e-5 relative L2 of the target overall, 2e-5 per field.
  Node-wise, a length-n FP32 dot product is off by at most n u sum|D||x|
  (n <= 165, u = 2^-24: 1e-5), 1e-3 after the amplification; the bar is
  5e-4 (measured up to 1.3e-4, node-per-thread kernel at acoustic N = 6; the
  oracle itself run in FP32 reaches 4.1e-5).
* Split 16-bit variants.  With a 16-bit unit roundoff v (2^-8 BF16, 2^-11
  FP16) the hi + lo pair holds an operand to v^2, and the dropped D_lo x_lo
  product is at most v^2 |D||x|, so each product carries up to about
  3 v^2 sum_m |D_nm||x_m|: 4.6e-5 of it for BF16, 7.2e-7 for FP16.
  FP16 is held to the 1e-4 target overall and per field, 2e-3 node-wise.
  BF16 cannot meet the target on these meshes: after the amplification its
  bound is ~5e-3 node-wise, and it measures 2e-5 .. 3.4e-4 relative L2
  (above 1e-4 for elastic N >= 4 and acoustic N >= 5).  It is held to its
  own bound (1e-3 overall and per field, 1e-2 node-wise); the benchmark's
  mixed form admits a split variant only where its right-hand side meets
  the 1e-4 target, which leaves BF16 out at those degrees.

A wrong element or face shows up at O(1) relative error node-wise, far
above every bar.
"""

import pytest
import torch

import dginputs as di
from tests._cases import Case, log

pytestmark = pytest.mark.gpu

FP32 = ("valu", "mfma", "elem")
SPLIT16 = ("mfma_bf16", "mfma_f16")
# (overall relative L2, per-field relative L2, node-wise) bars, derived above
BARS = {v: (1e-5, 2e-5, 5e-4) for v in FP32}
BARS["mfma_f16"] = (1e-4, 1e-4, 2e-3)
BARS["mfma_bf16"] = (1e-3, 1e-3, 1e-2)


def _variants(solver):
    from paper_1602_07997_amd._native import DG_E_UNSUPPORTED, DGError

    out = []
    for v in FP32 + SPLIT16:
        try:
            solver.variant = v
        except DGError as e:
            assert e.status == DG_E_UNSUPPORTED
            continue
        out.append(v)
    return out


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("N", list(range(1, 9)))
def test_paper_scale_rhs(physics, N):
    n = di.paper_scale_n(N)
    log(f"paper-scale rhs {physics} N={N} n={n}")
    mesh = di.kuhn_box(n, jitter=0.1, seed=0)
    kind = "layers" if physics == "acoustic" else "random"
    c = Case(physics, N, n, coef_kind=kind, init="pulses", mesh=mesh, seed=0)
    assert c.mesh.K == 6 * n ** 3
    ref = c.oracle.rhs(c.q0)
    q = c.to_gpu(c.q0_gpu)
    for v in _variants(c.solver):
        c.solver.variant = v
        r = c.to_host(c.solver.rhs(q))
        torch.cuda.synchronize()
        l2, pf, nd = BARS[v]
        err, _, _ = c.check(r, ref, l2, f"{v} K={c.mesh.K}", per_field=pf, node=nd)
        if v in SPLIT16:
            log(f"  {v}: {'meets' if err <= 1e-4 else 'misses'} the 1e-4 target")
