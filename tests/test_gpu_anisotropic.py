"""Anisotropic elasticity on the GPU against the FP64 oracle (C ABI).

The oracle's AnisotropicElasticOracle is pinned on the CPU (isotropic limit,
exact PDE right-hand side of polynomial states, energy rate, continuous
energy, plane-wave convergence).  Here the node-per-thread kernel of the
anisotropic physics runs on random heterogeneous media (a seeded symmetric
perturbation of an isotropic stiffness per element, float32-rounded for
both sides) with walls, absorbing faces and periodic faces of every
orientation.  Bars as for the isotropic physics: one right-hand side 2e-6
(relative L2, mass-weighted), 20 AB3 steps 1e-5, energy 1e-9.
"""

import numpy as np
import pytest
import torch

from oracle.dg import AB3Stepper
from oracle.multirate import TwoRateAB3
from paper_1602_07997_amd import _native as nat
from tests._cases import Case, log

import dginputs as di

pytestmark = pytest.mark.gpu

DEGREES = list(range(1, 9))


def _mesh_n(N):
    return 3 if N <= 4 else 2


@pytest.mark.parametrize("variant", ["valu", "mfma"])
@pytest.mark.parametrize("N", DEGREES)
def test_rhs_parity(N, variant):
    log(f"anisotropic rhs parity N={N} {variant}")
    c = Case("anisotropic", N, _mesh_n(N), jitter=0.1, seed=N, coef_kind="random", init="smooth")
    c.solver.variant = variant
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    c.check(c.to_host(r), c.oracle.rhs(c.q0), 2e-6, "rhs")


@pytest.mark.parametrize("variant", ["valu", "mfma"])
@pytest.mark.parametrize("N", [2, 5])
def test_rhs_parity_absorbing_faces(N, variant):
    log(f"anisotropic rhs parity, half the walls absorbing, N={N} {variant}")
    c = Case("anisotropic", N, 2, jitter=0.1, seed=50 + N, coef_kind="random", init="smooth", absorbing="half")
    c.solver.variant = variant
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    c.check(c.to_host(r), c.oracle.rhs(c.q0), 2e-6, "rhs absorbing")


@pytest.mark.parametrize("variant,N,periodic", [("valu", 1, True), ("valu", 3, False), ("valu", 4, True),
                                               ("mfma", 2, True), ("mfma", 6, False), ("mfma", 8, False)])
def test_all_face_orientations_parity(variant, N, periodic):
    """Vertices listed in random even orders, so that shared faces meet under
    all six relative orientations: one right-hand side and 20 AB3 steps."""
    log(f"anisotropic all orientations {variant} N={N} periodic={periodic}")
    mesh = di.relabel_vertices(di.kuhn_box(3, 2, 3, jitter=0.1, seed=60 + N, periodic=periodic), seed=70 + N)
    c = Case("anisotropic", N, 0, coef_kind="random", init="smooth", mesh=mesh, seed=60 + N)
    c.solver.variant = variant
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    c.check(c.to_host(r), c.oracle.rhs(c.q0), 2e-6, "rhs")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(20, c.dt)
    c.check(c.to_host(c.solver.get_fields()), AB3Stepper(c.oracle, c.q0).step(20, c.dt), 1e-5, "20 steps")


@pytest.mark.parametrize("variant", ["valu", "mfma"])
@pytest.mark.parametrize("N", DEGREES)
def test_steps_parity(N, variant):
    log(f"anisotropic 20-step parity N={N} {variant}")
    c = Case("anisotropic", N, _mesh_n(N), jitter=0.1, seed=10 + N, coef_kind="random", init="gaussian")
    c.solver.variant = variant
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(20, c.dt)
    q = c.to_host(c.solver.get_fields())
    c.check(q, AB3Stepper(c.oracle, c.q0).step(20, c.dt), 1e-5, "20 steps")


@pytest.mark.parametrize("N", [1, 3, 7, 8])
def test_energy_parity(N):
    log(f"anisotropic energy parity N={N}")
    c = Case("anisotropic", N, _mesh_n(N), jitter=0.1, seed=30 + N, coef_kind="random", init="smooth")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    e = c.solver.energy()
    e_ref = c.oracle.energy(c.q0)
    log(f"  energy {e:.12e} oracle {e_ref:.12e}")
    assert abs(e - e_ref) <= 1e-9 * e_ref


def test_energy_decays_over_a_run():
    """Upwind flux, walls: the discrete energy after the start-up steps does
    not grow over 60 steps of the stable time step."""
    c = Case("anisotropic", 3, 2, jitter=0.1, seed=71, coef_kind="random", init="gaussian")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(2, c.dt)
    e_prev = e0 = c.solver.energy()
    for _ in range(6):
        c.solver.step(10, c.dt)
        e = c.solver.energy()
        assert e <= e_prev * (1.0 + 1e-6)
        e_prev = e
    assert e_prev < e0


def test_two_rate_parity():
    """Two wave-speed layers (stiffness scaled by 4 on one side), fast class
    first: dg_step_multirate against the oracle's two-rate AB3."""
    from paper_1602_07997_amd import DGSolver
    from oracle.dg import make_oracle
    from oracle.mesh import build_mesh

    N = 2
    mesh = di.kuhn_box(3, jitter=0.1, seed=11)
    coef = di.anisotropic_random(mesh, seed=12)
    cen = di.element_centroids(mesh)
    coef[cen[:, 0] < 0.5, 1:] *= 4.0
    coef = coef.astype(np.float32).astype(np.float64)
    fast, dt = di.two_rate_classes(mesh, N, di.element_wave_speeds(coef, "anisotropic"))
    order = np.argsort(~fast, kind="stable")
    mesh = di.permute_elements(mesh, order)
    coef, fast = coef[order], fast[order]
    k_fast = int(fast.sum())
    assert 0 < k_fast < mesh.K
    geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo)
    s = DGSolver("anisotropic", N, mesh.elem_xyz, mesh.elem_topo)
    s.set_coefficients(torch.tensor(coef, dtype=torch.float32, device="cuda"))
    q0 = np.ascontiguousarray(np.moveaxis(di.gaussian_pulses(geo.xyz, 9, sigma=0.15), 0, 1))
    q0 = q0.astype(np.float32).astype(np.float64)
    s.set_rate_classes(k_fast)
    s.set_fields(torch.tensor(q0, dtype=torch.float32, device="cuda"))
    s.step_multirate(20, dt)
    o = make_oracle("anisotropic", geo, coef)
    ref = TwoRateAB3(o, q0, fast).macro_step(20, dt)
    from tests._cases import check_close

    check_close(o, s.get_fields().double().cpu().numpy(), ref, 1e-5, "two-rate 20 macro steps")
    s.close()


def test_batch_member_matches_alone():
    from paper_1602_07997_amd import DGBatch, DGSolver

    specs = ((2, (3, 2, 2), "valu"), (3, (2, 3, 2), "valu"), (5, (2, 2, 2), "mfma"))
    cases = [Case("anisotropic", N, None, jitter=0.1, seed=80 + N, coef_kind="random", init="gaussian", dims=d)
             for N, d, _ in specs]
    twins = []
    for c, (_, _, v) in zip(cases, specs):
        c.solver.variant = v
        c.solver.set_fields(c.to_gpu(c.q0_gpu))
        t = DGSolver("anisotropic", c.N, c.mesh.elem_xyz, c.mesh.elem_topo)
        t.variant = v
        t.set_coefficients(torch.tensor(c.coef, dtype=torch.float32, device="cuda"))
        t.set_fields(c.to_gpu(c.q0_gpu))
        twins.append(t)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    b = DGBatch([c.solver for c in cases], stream=stream)
    b.step(12, [c.dt for c in cases])
    for c, t in zip(cases, twins):
        t.step(12, c.dt)
    stream.synchronize()
    torch.cuda.synchronize()
    for c, t in zip(cases, twins):
        assert torch.equal(c.solver.get_fields(), t.get_fields())
        c.check(c.to_host(c.solver.get_fields()), AB3Stepper(c.oracle, c.q0).step(12, c.dt), 1e-5, "batch member")
    b.close()


def test_invalid_stiffness_is_refused():
    c = Case("anisotropic", 2, 2, jitter=0.1, seed=90, coef_kind="random", init="gaussian")
    good = torch.tensor(c.coef, dtype=torch.float32, device="cuda")
    for k, what in ((3, "indefinite"), (7, "density"), (11, "nan")):
        bad = good.clone()
        if what == "indefinite":
            bad[k, 1] = -1.0  # C_00 < 0
        elif what == "density":
            bad[k, 0] = 0.0
        else:
            bad[k, 9] = float("nan")
        with pytest.raises(nat.DGError) as ei:
            c.solver.set_coefficients(bad)
        assert ei.value.status == nat.DG_E_ARG
        assert f"element {k}" in str(ei.value)
    # no coefficients now: stepping is refused until valid ones arrive
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    with pytest.raises(nat.DGError) as ei:
        c.solver.step(1, c.dt)
    assert ei.value.status == nat.DG_E_STATE
    c.solver.set_coefficients(good)
    c.solver.step(1, c.dt)


def test_only_valu_and_fp32_mfma_and_no_misfit_are_built():
    from paper_1602_07997_amd import DGMisfit

    c = Case("anisotropic", 3, 2, jitter=0.1, seed=91, coef_kind="random", init="gaussian")
    for v in ("mfma_bf16", "mfma_f16", "elem", "mfma_wide"):
        with pytest.raises(nat.DGError) as ei:
            c.solver.variant = v
        assert ei.value.status == nat.DG_E_UNSUPPORTED
    assert c.solver.variant == "valu"
    c.solver.variant = "mfma"
    assert c.solver.variant == "mfma"
    with pytest.raises(nat.DGError) as ei:
        DGMisfit(c.solver, 10, c.dt, [[0.5, 0.5, 0.5]], np.zeros(11), [[0.3, 0.4, 0.5]])
    assert ei.value.status == nat.DG_E_UNSUPPORTED
