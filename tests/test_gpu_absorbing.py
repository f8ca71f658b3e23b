"""Absorbing boundary faces on the GPU against the FP64 oracle (C ABI).

Absorbing faces see a zero exterior state with the element's own
coefficients (the oracle's pins: outgoing plane waves exact, boundary
dissipation equal to the characteristic flux, a pulse leaving the box).
Every kernel variant of both physics takes the same ghost state from bit 3
of a wall's connectivity word; the cases mix absorbing and reflecting walls
(a seeded half of the unpaired faces) so that both paths run in one launch.
Bars as in the other parity tests: one right-hand side 2e-6, 20 AB3 steps
1e-5 (FP32 variants); the FP16 split variant 1e-4.  The misfit gradient on
a mesh with absorbing faces is checked against the oracle's complex-step
gradient (2e-4), which rests on the transpose identity pinned for absorbing
faces on assembled operators.
"""

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.dg import AB3Stepper, make_oracle
from oracle.mesh import build_mesh
from paper_1602_07997_amd import _native as nat
from tests._cases import Case, coefficients, log

pytestmark = pytest.mark.gpu

CASES = (
    [("acoustic", N, v) for N in (1, 2, 3, 5, 8) for v in ("valu", "mfma", "mfma_f16")]
    + [("elastic", N, v) for N in (1, 2, 4, 6, 8) for v in ("valu", "mfma", "mfma_f16")]
    + [("acoustic", 1, "elem"), ("acoustic", 2, "elem"), ("elastic", 1, "elem")]
)


def _try_variant(s, v):
    try:
        s.variant = v
    except nat.DGError as e:
        assert e.status == nat.DG_E_UNSUPPORTED
        return False
    return True


@pytest.mark.parametrize("physics,N,variant", CASES)
def test_absorbing_parity(physics, N, variant):
    n = 3 if N <= 4 else 2
    # a smooth state that is O(1) on the boundary, so that the walls matter
    c = Case(physics, N, n, jitter=0.1, seed=30 + N, coef_kind="random", init="smooth", absorbing="half")
    assert _try_variant(c.solver, variant)
    log(f"absorbing parity {physics} N={N} {variant}: {int(c.absorbing.sum())} of {int(c.geo.wall.sum())} walls")
    l2_rhs, l2_steps = (2e-6, 1e-5) if variant != "mfma_f16" else (1e-4, 1e-4)
    q = c.to_gpu(c.q0_gpu)
    c.check(c.to_host(c.solver.rhs(q)), c.oracle.rhs(c.q0), l2_rhs, "rhs")
    c.solver.set_fields(q)
    c.solver.step(20, c.dt)
    ref = AB3Stepper(c.oracle, c.q0).step(20, c.dt)
    c.check(c.to_host(c.solver.get_fields()), ref, l2_steps, "20 steps")
    e_gpu, e_ref = c.solver.energy(), c.oracle.energy(ref)
    assert abs(e_gpu - e_ref) <= 1e-5 * e_ref


def test_boundary_kinds_validated():
    c = Case("acoustic", 2, 2, jitter=0.1, seed=3, coef_kind="random", init="gaussian")
    bad = np.zeros((c.mesh.K, 4), dtype=bool)
    k, f = np.nonzero(~c.geo.wall)
    bad[k[0], f[0]] = True  # a face with a neighbour
    with pytest.raises(nat.DGError) as ei:
        c.solver.set_boundary(bad)
    assert ei.value.status == nat.DG_E_ARG
    # the refused call changed nothing: walls still reflect
    conn = c.solver.debug_buffer("conn").reshape(c.mesh.K, 4)
    assert np.all(conn[c.geo.wall] & 15 == 7)
    c.solver.set_boundary(c.geo.wall)
    conn = c.solver.debug_buffer("conn").reshape(c.mesh.K, 4)
    kk = np.nonzero(c.geo.wall)[0]
    assert np.array_equal(conn[c.geo.wall], (kk << 5) | 15)
    c.solver.set_boundary(np.zeros((c.mesh.K, 4), dtype=bool))
    conn = c.solver.debug_buffer("conn").reshape(c.mesh.K, 4)
    assert np.array_equal(conn[c.geo.wall], (kk << 5) | 7)


def test_pulse_leaves_the_box():
    """A right-going acoustic pulse on a slab open along x: the GPU matches the
    oracle while the pulse crosses the outflow face, and after it has crossed
    less than 1e-6 of its energy is left (a rigid wall keeps it all)."""
    from paper_1602_07997_amd import DGSolver

    N = 3
    m = di.kuhn_box(10, 3, 3, jitter=0.0, periodic=(False, True, True))
    geo = build_mesh(N, m.elem_xyz, m.elem_topo, m.period)
    coef = np.tile([1.0, 1.0], (geo.K, 1))
    s = DGSolver("acoustic", N, m.elem_xyz, m.elem_topo)
    s.set_coefficients(torch.tensor(coef, dtype=torch.float32, device="cuda"))
    s.set_boundary(geo.wall)

    def pulse(x):
        g = np.exp(-((x[..., 0] - 0.5) ** 2) / (2 * 0.08**2))
        q = np.zeros(x.shape[:-1] + (4,))
        q[..., 0] = g
        q[..., 1] = g
        return np.ascontiguousarray(np.moveaxis(q, -1, 1)).astype(np.float32)

    q0 = pulse(s.node_coordinates())
    s.set_fields(torch.tensor(q0, device="cuda"))
    e0 = s.energy()
    dt = di.time_step(m, N, 1.0)
    n_half = int(np.ceil(0.6 / dt))  # the pulse is half way through the face
    s.step(n_half, dt)
    o = make_oracle("acoustic", geo, coef, absorbing=geo.wall)
    ref = AB3Stepper(o, pulse(geo.xyz).astype(np.float64)).step(n_half, dt)
    got = s.get_fields().double().cpu().numpy()
    err, _ = o.rel_l2(got, ref)
    log(f"  pulse half way out: rel L2 {err:.2e}, energy left {s.energy() / e0:.3e}")
    assert err <= 1e-5
    assert abs(s.energy() - o.energy(ref)) <= 1e-5 * o.energy(ref)
    s.step(int(np.ceil(1.0 / dt)) - n_half, dt)
    assert s.energy() / e0 < 1e-6
    s.close()


@pytest.mark.parametrize("physics,N", [("acoustic", 2), ("elastic", 2)])
def test_gradient_with_absorbing_faces(physics, N):
    from oracle.misfit import MisfitProblem
    from paper_1602_07997_amd import DGMisfit, DGSolver

    mesh = di.kuhn_box(2, 2, 2, jitter=0.1, seed=3)
    coef = coefficients(physics, mesh, "random", 5)
    dt = di.time_step(mesh, N, di.max_wave_speed(coef, physics))
    steps = 30
    geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo)
    absorbing = geo.wall & (np.random.default_rng(4).random(geo.wall.shape) < 0.5)
    rng = np.random.default_rng(0)
    src = np.array([0.5, 0.45, 0.55])
    rec = rng.uniform(0.1, 0.9, (4, 3))
    pr = MisfitProblem(physics, geo, mesh.elem_xyz, dt, steps, src, rec, f0=3.0, t0=0.3, absorbing=absorbing)
    coef2 = (coef * (1 + 0.05 * rng.standard_normal(coef.shape))).astype(np.float32).astype(np.float64)
    data = pr.forward(coef2)
    s = DGSolver(physics, N, mesh.elem_xyz, mesh.elem_topo)
    s.set_boundary(absorbing)
    s.set_coefficients(torch.tensor(coef, dtype=torch.float32, device="cuda"))
    f = DGMisfit(s, steps, dt, src, pr.wavelet, rec, checkpoint_every=7)
    f.forward(torch.tensor(data, dtype=torch.float32, device="cuda"))
    g = f.gradient().double().cpu().numpy()
    g_ref = pr.gradient_complex_step(coef, data)
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    worst = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    log(f"  absorbing gradient {physics} N={N}: rel L2 {err:.2e}, max {worst:.2e}")
    assert err <= 2e-4 and worst <= 2e-4
    f.close()
    s.close()
