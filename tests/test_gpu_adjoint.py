"""Misfit and coefficient gradient on the GPU against the FP64 oracle.

* receiver traces of the forward solve with a point source: relative L2
  <= 1e-5 against the oracle's traces (the AB3 tolerance);
* gradient by the GPU discrete adjoint against the oracle's complex-step
  gradient: relative L2 over all coefficients <= 2e-4 and every entry within
  2e-4 of the largest (FP32 states, FP64 accumulation);
* the checkpoint interval changes nothing (the recomputed segments are the
  same kernels on the same inputs: identical results);
* at the paper-scale adjoint workload (elastic N=4, 14,196 tetrahedra, 200
  steps, checkpoints every 20) central differences of the FP32 GPU misfit
  agree with the gradient to 5e-3 on the 8 most sensitive coefficients (the
  FP32 rounding of J over the 0.2% step bounds the differences; exactness is
  the complex-step comparison above).
"""

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.mesh import build_mesh
from oracle.misfit import MisfitProblem, locate
from tests._cases import coefficients, log

pytestmark = pytest.mark.gpu


def _setup(physics, N, steps=30, ckpt=7, dims=(2, 2, 2), seed=5, relabel=False):
    from paper_1602_07997_amd import DGMisfit, DGSolver

    mesh = di.kuhn_box(*dims, jitter=0.1, seed=3)
    if relabel:  # random even vertex orders: shared faces meet in all six orientations
        mesh = di.relabel_vertices(mesh, seed=6)
    coef = coefficients(physics, mesh, "random", seed)
    dt = di.time_step(mesh, N, di.max_wave_speed(coef, physics))
    rng = np.random.default_rng(0)
    src = np.array([0.5, 0.45, 0.55])
    rec = rng.uniform(0.1, 0.9, (4, 3))
    geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo)
    pr = MisfitProblem(physics, geo, mesh.elem_xyz, dt, steps, src, rec, f0=3.0, t0=0.3)
    coef2 = (coef * (1 + 0.05 * rng.standard_normal(coef.shape))).astype(np.float32).astype(np.float64)
    data = pr.forward(coef2)
    s = DGSolver(physics, N, mesh.elem_xyz, mesh.elem_topo)
    s.set_coefficients(torch.tensor(coef, dtype=torch.float32, device="cuda"))
    f = DGMisfit(s, steps, dt, src, pr.wavelet, rec, checkpoint_every=ckpt)
    return mesh, coef, pr, data, s, f


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_locate_points_matches_oracle(physics):
    from paper_1602_07997_amd import DGSolver

    mesh = di.kuhn_box(3, 2, 2, jitter=0.15, seed=4)
    s = DGSolver(physics, 3, mesh.elem_xyz, mesh.elem_topo)
    x = np.random.default_rng(1).uniform(0.05, 0.95, (20, 3))
    k, w = s.locate_points(x)
    k_ref, _ = locate(mesh.elem_xyz, x)
    assert np.array_equal(k, k_ref)
    # weights reproduce the node coordinates' linear functions at x
    xyz = s.node_coordinates()
    np.testing.assert_allclose(np.einsum("pn,pni->pi", w, xyz[k]), x, atol=1e-12)


@pytest.mark.parametrize("physics,N", [("acoustic", 2), ("acoustic", 3), ("elastic", 2)])
def test_misfit_forward_matches_oracle(physics, N):
    log(f"misfit forward {physics} N={N}")
    _, coef, pr, data, s, f = _setup(physics, N)
    traces, J = f.forward(torch.tensor(data, dtype=torch.float32, device="cuda"))
    u = traces.double().cpu().numpy()
    u_ref = pr.forward(coef)
    err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    J_ref = pr.misfit(coef, data)
    log(f"  traces rel L2 {err:.2e}; J {J:.6e} vs {J_ref:.6e}")
    assert err <= 1e-5
    assert J == pytest.approx(J_ref, rel=1e-3)


def test_misfit_refuses_the_fp16_split_variant():
    """The projected point source exceeds FP16's range, so a solver on the
    FP16 split products gets DG_E_UNSUPPORTED from the misfit calls (the
    BF16 split, with FP32's exponent range, runs)."""
    from paper_1602_07997_amd import _native as nat

    _, coef, pr, data, s, f = _setup("acoustic", 2, steps=10)
    d = torch.tensor(data[: 11], dtype=torch.float32, device="cuda")
    s.variant = "mfma_f16"
    with pytest.raises(nat.DGError) as ei:
        f.forward(d)
    assert ei.value.status == nat.DG_E_UNSUPPORTED
    s.variant = "mfma_bf16"
    _, J = f.forward(d)
    assert np.isfinite(J) and J > 0.0
    s.variant = "mfma_f16"
    with pytest.raises(nat.DGError) as ei:
        f.gradient()
    assert ei.value.status == nat.DG_E_UNSUPPORTED
    s.variant = "valu"
    assert np.all(np.isfinite(f.gradient().cpu().numpy()))


@pytest.mark.parametrize("physics,N", [("acoustic", 2), ("acoustic", 3), ("elastic", 2), ("elastic", 3)])
def test_gradient_matches_complex_step(physics, N):
    log(f"adjoint gradient {physics} N={N}")
    _, coef, pr, data, s, f = _setup(physics, N)
    f.forward(torch.tensor(data, dtype=torch.float32, device="cuda"))
    g = f.gradient().double().cpu().numpy()
    g_ref = pr.gradient_complex_step(coef, data)
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    worst = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    log(f"  rel L2 {err:.2e}, max {worst:.2e}")
    assert err <= 2e-4 and worst <= 2e-4


@pytest.mark.parametrize("physics,N", [("acoustic", 3), ("elastic", 2)])
def test_gradient_all_face_orientations(physics, N):
    log(f"adjoint gradient, relabelled vertices, {physics} N={N}")
    _, coef, pr, data, s, f = _setup(physics, N, relabel=True)
    f.forward(torch.tensor(data, dtype=torch.float32, device="cuda"))
    g = f.gradient().double().cpu().numpy()
    g_ref = pr.gradient_complex_step(coef, data)
    err = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    worst = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    log(f"  rel L2 {err:.2e}, max {worst:.2e}")
    assert err <= 2e-4 and worst <= 2e-4


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_checkpoint_interval_changes_nothing(physics):
    from paper_1602_07997_amd import DGMisfit

    _, coef, pr, data, s, f = _setup(physics, 2, steps=23, ckpt=1)
    d = torch.tensor(data, dtype=torch.float32, device="cuda")
    outs = []
    for ckpt in (1, 5, 23, 40):
        f = DGMisfit(s, 23, pr.dt, [0.5, 0.45, 0.55], pr.wavelet, np.random.default_rng(0).uniform(0.1, 0.9, (4, 3)),
                     checkpoint_every=ckpt)
        tr, J = f.forward(d)
        outs.append((tr, J, f.gradient()))
        f.close()
    for tr, J, g in outs[1:]:
        assert torch.equal(tr, outs[0][0]) and J == outs[0][1] and torch.equal(g, outs[0][2])
    # a second gradient call (all segments recomputed) gives the same result
    f = DGMisfit(s, 23, pr.dt, [0.5, 0.45, 0.55], pr.wavelet, np.random.default_rng(0).uniform(0.1, 0.9, (4, 3)),
                 checkpoint_every=5)
    f.forward(d)
    g1 = f.gradient()
    g2 = f.gradient()
    assert torch.equal(g1, g2) and torch.equal(g1, outs[0][2])


def test_autograd_function():
    from paper_1602_07997_amd import misfit

    _, coef, pr, data, s, f = _setup("acoustic", 2)
    d = torch.tensor(data, dtype=torch.float32, device="cuda")
    c = torch.tensor(coef, dtype=torch.float32, device="cuda", requires_grad=True)
    J = misfit(c, f, d)
    (3.0 * J).backward()
    _, J2 = f.forward(d)
    g = f.gradient()
    assert float(J) == pytest.approx(J2)
    torch.testing.assert_close(c.grad, 3.0 * g)


def test_autograd_interleaved_forwards_and_coefficient_changes():
    """Two misfit evaluations (a line search, or a sum of two misfits) before
    one backward: each gradient belongs to its own call's coefficients, and
    the solver's coefficients are left as they were.  At the ABI level a
    gradient after a coefficient change is refused."""
    from paper_1602_07997_amd import misfit
    from paper_1602_07997_amd._native import DG_E_STATE, DGError

    _, coef, pr, data, s, f = _setup("acoustic", 2)
    d = torch.tensor(data, dtype=torch.float32, device="cuda")
    c1 = torch.tensor(coef, dtype=torch.float32, device="cuda", requires_grad=True)
    c2 = torch.tensor(coef * 1.03, dtype=torch.float32, device="cuda", requires_grad=True)
    # reference gradients, one call at a time
    misfit(c1, f, d).backward()
    g1_ref = c1.grad.clone()
    misfit(c2, f, d).backward()
    g2_ref = c2.grad.clone()
    assert not torch.allclose(g1_ref, g2_ref)
    c1.grad = None
    c2.grad = None
    J = misfit(c1, f, d) + 2.0 * misfit(c2, f, d)
    J.backward()
    torch.testing.assert_close(c1.grad, g1_ref)
    torch.testing.assert_close(c2.grad, 2.0 * g2_ref)
    # the solver's coefficients are those of the last forward call (c2)
    torch.testing.assert_close(s.last_coefficients, c2.detach())
    # ABI: forward, coefficient change, gradient -> DG_E_STATE
    f.forward(d)
    s.set_coefficients(c1.detach())
    with pytest.raises(DGError) as ei:
        f.gradient()
    assert ei.value.status == DG_E_STATE


def test_paper_scale_adjoint_finite_differences():
    """Elastic N=4 on the 13x13x14 Kuhn box (14,196 tetrahedra), 200 steps,
    checkpoints every 20, Ricker source (peak frequency 5) at the box centre,
    64 receivers uniform in [0.1, 0.9]^3 (seed 4), data from coefficients
    with a +5% Gaussian blob; central differences of the GPU misfit on the
    8 coefficients of largest sensitivity |g c| (the sensitivity falls off
    steeply away from the source and receivers: only 3 coefficients reach a
    quarter of the largest, and below that the FP32 rounding of J swamps a
    0.2% central difference).  200 CFL-limited
    steps span a small part of one period of the wavelet, so its peak is
    placed in the middle of the window (t0 = 100 dt)."""
    from paper_1602_07997_amd import DGMisfit, DGSolver
    from paper_1602_07997_amd.adjoint import ricker

    log("paper-scale adjoint: elastic N=4, 14196 tets, 200 steps")
    N, steps = 4, 200
    mesh = di.kuhn_box(13, 13, 14, jitter=0.1, seed=3)
    assert mesh.K == 14196
    coef = di.elastic_loguniform(mesh, 3).astype(np.float32).astype(np.float64)
    dt = di.time_step(mesh, N, di.max_wave_speed(coef, "elastic"))
    rec = np.random.default_rng(4).uniform(0.1, 0.9, (64, 3))
    src = np.array([0.5, 0.5, 0.5])
    wav = ricker(np.arange(steps + 1) * dt, 5.0, 0.5 * steps * dt)
    cen = di.element_centroids(mesh)
    blob = 1.0 + 0.05 * np.exp(-np.sum((cen - np.array([0.35, 0.6, 0.5])) ** 2, 1) / (2 * 0.15 ** 2))
    coef2 = coef * blob[:, None]
    s = DGSolver("elastic", N, mesh.elem_xyz, mesh.elem_topo)
    f = DGMisfit(s, steps, dt, src, wav, rec, checkpoint_every=20)
    s.set_coefficients(torch.tensor(coef2, dtype=torch.float32, device="cuda"))
    data, _ = f.forward()
    ct = torch.tensor(coef, dtype=torch.float32, device="cuda")
    s.set_coefficients(ct)
    _, J = f.forward(data)
    g = f.gradient().double().cpu().numpy()
    log(f"  J = {J:.6e}, |g| max {np.abs(g).max():.3e}")
    assert J > 0.0
    sens = np.abs(g * coef).ravel()
    flat = np.argsort(sens)[::-1][:8]
    results = []
    for idx in flat:
        k, p = np.unravel_index(idx, g.shape)
        h = 2e-3 * coef[k, p]
        vals, cs = [], []
        for sgn in (1.0, -1.0):
            c2 = coef.copy()
            c2[k, p] += sgn * h
            c2 = c2.astype(np.float32)
            cs.append(float(c2[k, p]))  # the perturbation the GPU actually sees
            s.set_coefficients(torch.tensor(c2, device="cuda"))
            vals.append(f.forward(data)[1])
        fd = (vals[0] - vals[1]) / (cs[0] - cs[1])
        log(f"  k={k} p={p}: adjoint {g[k, p]:.6e} fd {fd:.6e} rel {abs(fd - g[k, p]) / abs(g[k, p]):.1e}")
        results.append((fd, g[k, p]))
    s.set_coefficients(ct)
    for fd, ga in results:
        assert fd == pytest.approx(ga, rel=5e-3)
