"""Two-rate (local) time stepping on the GPU against the FP64 oracle (C ABI).

The oracle's TwoRateAB3 is pinned on the CPU (dense-output weights, single
class = single-rate AB3 bit for bit, third-order convergence, energy).  Here
every kernel variant of both physics runs dg_step_multirate on meshes whose
elements are ordered fast class first: two wave-speed layers (c = 2 | 1)
and a size-graded mesh.  Bars: 30 macro steps 1e-5 relative L2 (FP32
variants), 1e-4 (FP16 split).  With one class the two-rate path is the
single-rate path bit for bit (the same kernels on the same data).
"""

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.dg import make_oracle
from oracle.mesh import build_mesh
from oracle.multirate import TwoRateAB3
from paper_1602_07997_amd import _native as nat
from tests._cases import check_close, log

pytestmark = pytest.mark.gpu


def _case(physics, N, graded=False):
    from paper_1602_07997_amd import DGSolver

    if graded:
        mesh = di.graded_kuhn_box(5, 2)
        coef = np.tile([1.0, 1.0], (mesh.K, 1)) if physics == "acoustic" else np.tile([1.0, 1.0, 1.0], (mesh.K, 1))
    else:
        mesh = di.kuhn_box(3, jitter=0.1, seed=11)
        cen = di.element_centroids(mesh)
        if physics == "acoustic":
            coef = np.where(cen[:, :1] < 0.5, [[1.0, 2.0]], [[1.2, 1.0]])
        else:
            coef = np.where(cen[:, :1] < 0.5, [[1.0, 2.0, 1.5]], [[1.1, 0.5, 0.375]])
    coef = coef.astype(np.float32).astype(np.float64)
    fast, dt = di.two_rate_classes(mesh, N, di.element_wave_speeds(coef, physics))
    order = np.argsort(~fast, kind="stable")  # fast class first
    mesh = di.permute_elements(mesh, order)
    coef, fast = coef[order], fast[order]
    k_fast = int(fast.sum())
    assert np.all(fast[:k_fast]) and not np.any(fast[k_fast:])
    geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo)
    s = DGSolver(physics, N, mesh.elem_xyz, mesh.elem_topo)
    s.set_coefficients(torch.tensor(coef, dtype=torch.float32, device="cuda"))
    nf = 4 if physics == "acoustic" else 9
    q0 = np.ascontiguousarray(np.moveaxis(di.gaussian_pulses(geo.xyz, nf, sigma=0.15), 0, 1))
    q0 = q0.astype(np.float32).astype(np.float64)
    return mesh, geo, coef, fast, k_fast, dt, q0, s


CASES = (
    [("acoustic", N, v) for N in (2, 3, 5) for v in ("valu", "mfma", "mfma_f16")]
    + [("elastic", N, v) for N in (2, 4) for v in ("valu", "mfma", "mfma_f16")]
    + [("acoustic", 2, "elem")]
)


@pytest.mark.parametrize("physics,N,variant", CASES)
def test_two_rate_parity(physics, N, variant):
    mesh, geo, coef, fast, k_fast, dt, q0, s = _case(physics, N)
    log(f"two-rate {physics} N={N} {variant}: {k_fast} fast of {geo.K}, dt {dt:.3e}")
    s.variant = variant
    s.set_rate_classes(k_fast)
    s.set_fields(torch.tensor(q0, dtype=torch.float32, device="cuda"))
    s.step_multirate(30, dt)
    got = s.get_fields().double().cpu().numpy()
    o = make_oracle(physics, geo, coef)
    ref = TwoRateAB3(o, q0, fast).macro_step(30, dt)
    check_close(o, got, ref, 1e-5 if variant != "mfma_f16" else 1e-4, "30 macro steps")
    assert s.step_index == 30
    s.close()


def test_two_rate_parity_graded_mesh():
    mesh, geo, coef, fast, k_fast, dt, q0, s = _case("acoustic", 3, graded=True)
    log(f"two-rate graded: {k_fast} fast of {geo.K}")
    assert 0 < k_fast < geo.K
    s.variant = "mfma"
    s.set_rate_classes(k_fast)
    s.set_fields(torch.tensor(q0, dtype=torch.float32, device="cuda"))
    s.step_multirate(25, dt)
    o = make_oracle("acoustic", geo, coef)
    ref = TwoRateAB3(o, q0, fast).macro_step(25, dt)
    check_close(o, s.get_fields().double().cpu().numpy(), ref, 1e-5, "graded 25 macro steps")
    s.close()


@pytest.mark.parametrize("k_fast", ["none", "all"])
def test_one_class_equals_single_rate_bitwise(k_fast):
    mesh, geo, coef, fast, _, dt, q0, s = _case("acoustic", 3)
    q = torch.tensor(q0, dtype=torch.float32, device="cuda")
    s.variant = "mfma"
    s.set_rate_classes(0 if k_fast == "none" else geo.K)
    s.set_fields(q)
    s.step_multirate(9, dt)
    got = s.get_fields().clone()
    s.set_rate_classes(0)
    s.set_fields(q)
    if k_fast == "none":
        s.step(9, dt)
    else:
        s.step(18, dt / 2)
    assert torch.equal(got, s.get_fields())
    s.close()


def test_two_rate_solver_refuses_single_rate_calls():
    mesh, geo, coef, fast, k_fast, dt, q0, s = _case("acoustic", 2)
    s.set_rate_classes(k_fast)
    s.set_fields(torch.tensor(q0, dtype=torch.float32, device="cuda"))
    with pytest.raises(nat.DGError) as ei:
        s.step(1, dt)
    assert ei.value.status == nat.DG_E_STATE
    with pytest.raises(nat.DGError) as ei:
        s.get_state()
    assert ei.value.status == nat.DG_E_UNSUPPORTED
    with pytest.raises(nat.DGError) as ei:
        s.set_rate_classes(geo.K + 1)
    assert ei.value.status == nat.DG_E_ARG
    s.close()


def test_two_rate_is_stable_where_single_rate_is_not():
    """On the two-layer acoustic case single-rate AB3 at the macro step blows
    up (the oracle shows it); the GPU two-rate run keeps a bounded, decaying
    energy over 200 macro steps."""
    mesh, geo, coef, fast, k_fast, dt, q0, s = _case("acoustic", 2)
    s.variant = "valu"
    s.set_rate_classes(k_fast)
    s.set_fields(torch.tensor(q0, dtype=torch.float32, device="cuda"))
    s.step_multirate(2, dt)
    e2 = s.energy()
    s.step_multirate(198, dt)
    assert s.energy() < e2
    s.close()
