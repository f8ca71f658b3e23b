"""Pins of the misfit oracle (point source, receivers, complex-step gradient)
and of the transpose identity the adjoint path is built on."""

import numpy as np
import pytest

import dginputs as di
from oracle.dg import make_oracle
from oracle.mesh import build_mesh
from oracle.misfit import MisfitProblem, lagrange_weights, locate, ricker
from oracle.refelem import reference_element, tet_basis_indices


def _poly(N, rng):
    """A random polynomial of total degree N in (r, s, t) and its evaluator."""
    terms = [(i, j, k) for i in range(N + 1) for j in range(N + 1 - i) for k in range(N + 1 - i - j)]
    c = rng.standard_normal(len(terms))

    def f(x):
        x = np.atleast_2d(x)
        return sum(ci * x[:, 0] ** i * x[:, 1] ** j * x[:, 2] ** k for ci, (i, j, k) in zip(c, terms))

    return f


@pytest.mark.parametrize("N", [1, 2, 4, 6])
def test_lagrange_weights_interpolate_degree_N_exactly(N):
    ref = reference_element(N)
    rng = np.random.default_rng(N)
    f = _poly(N, rng)
    # random points inside the reference tetrahedron
    lam = rng.dirichlet(np.ones(4), size=20)
    xi = np.stack([-1 + 2 * lam[:, 1], -1 + 2 * lam[:, 2], -1 + 2 * lam[:, 3]], 1)
    w = lagrange_weights(ref, xi)
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(w @ f(ref.r), f(xi), atol=1e-11 * max(1.0, np.abs(f(xi)).max()))
    # at the nodes the weights are the identity
    np.testing.assert_allclose(lagrange_weights(ref, ref.r), np.eye(ref.Np), atol=1e-11)
    assert len(tet_basis_indices(N)) == ref.Np


def test_locate_maps_points_back():
    mesh = di.kuhn_box(3, 2, 2, jitter=0.15, seed=4)
    rng = np.random.default_rng(1)
    x = rng.uniform(0.05, 0.95, (30, 3))
    k, xi = locate(mesh.elem_xyz, x)
    xv = mesh.elem_xyz[k]
    F = 0.5 * np.stack([xv[:, 1] - xv[:, 0], xv[:, 2] - xv[:, 0], xv[:, 3] - xv[:, 0]], -1)
    np.testing.assert_allclose(xv[:, 0] + np.einsum("pij,pj->pi", F, xi + 1.0), x, atol=1e-12)
    lam = np.concatenate([-(1 + xi.sum(1, keepdims=True)) / 2, (1 + xi) / 2], 1)
    assert np.all(lam >= -1e-12)
    with pytest.raises(ValueError):
        locate(mesh.elem_xyz, [[1.5, 0.5, 0.5]])


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_point_source_is_a_discrete_delta(physics):
    """J_k b^T M u = u(x_s) for every u of degree N: b is the Galerkin
    projection of the Dirac mass at the source point."""
    N = 3
    mesh = di.kuhn_box(2, 2, 2, jitter=0.1, seed=2)
    geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo)
    xs = np.array([0.41, 0.52, 0.37])
    pr = MisfitProblem(physics, geo, mesh.elem_xyz, 1e-3, 1, xs, [[0.5, 0.5, 0.5]], f0=3.0)
    rng = np.random.default_rng(3)
    f = _poly(N, rng)
    k = pr.src_elem[0]
    u = f(geo.xyz[k])
    c = pr.src_fields[0]
    got = geo.J[k] * pr.b[k, c] @ geo.ref.M @ u
    np.testing.assert_allclose(got, f(xs)[0], rtol=1e-10)
    # every other element and field is untouched
    mask = np.ones(pr.b.shape, bool)
    mask[k, list(pr.src_fields)] = False
    assert np.all(pr.b[mask] == 0.0)


def test_ricker_closed_form():
    f0, t0 = 5.0, 0.24
    assert ricker(t0, f0, t0) == pytest.approx(1.0)
    tz = 1.0 / (np.pi * f0 * np.sqrt(2.0))  # zero crossings at t0 +- tz
    assert abs(ricker(t0 + tz, f0, t0)) < 1e-15 and abs(ricker(t0 - tz, f0, t0)) < 1e-15
    tau = np.linspace(0, 0.3, 7)
    np.testing.assert_allclose(ricker(t0 + tau, f0, t0), ricker(t0 - tau, f0, t0))
    # minimum value -2 exp(-3/2) at t0 +- sqrt(3/2)/(pi f0)
    tm = np.sqrt(1.5) / (np.pi * f0)
    assert ricker(t0 + tm, f0, t0) == pytest.approx(-2.0 * np.exp(-1.5))


def _problem(physics, N=2, steps=30, seed=5):
    mesh = di.kuhn_box(2, 2, 2, jitter=0.1, seed=3)
    geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo)
    coef = di.acoustic_loguniform(mesh, seed) if physics == "acoustic" else di.elastic_loguniform(mesh, seed)
    dt = di.time_step(mesh, N, di.max_wave_speed(coef, physics))
    rng = np.random.default_rng(0)
    pr = MisfitProblem(physics, geo, mesh.elem_xyz, dt, steps, [0.5, 0.45, 0.55],
                       rng.uniform(0.1, 0.9, (4, 3)), f0=3.0, t0=0.3)
    coef2 = coef * (1 + 0.05 * rng.standard_normal(coef.shape))
    return pr, coef, pr.forward(coef2)


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_complex_step_matches_central_differences(physics):
    pr, coef, data = _problem(physics)
    elems = [33, 44]  # elements near the receivers, where the gradient is large
    g = pr.gradient_complex_step(coef, data, elems)
    for k in elems:
        for p in range(coef.shape[1]):
            h = 1e-6 * coef[k, p]
            cp, cm = coef.copy(), coef.copy()
            cp[k, p] += h
            cm[k, p] -= h
            fd = (pr.misfit(cp, data) - pr.misfit(cm, data)) / (2 * h)
            assert fd == pytest.approx(g[k, p], rel=1e-6)


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_misfit_vanishes_at_the_data(physics):
    pr, coef, other = _problem(physics, steps=12)
    data = pr.forward(coef)
    assert pr.misfit(coef, data) == 0.0
    g = pr.gradient_complex_step(coef, data, elems=[33, 44])
    scale = np.abs(pr.gradient_complex_step(coef, other, elems=[33, 44])).max()
    # zero up to the rounding of the complex-arithmetic forward solve
    assert np.abs(g).max() <= 1e-9 * scale


@pytest.mark.parametrize("absorbing", [False, True])
@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_transpose_identity(physics, absorbing):
    """A^T = P W A P W^{-1}: W the energy weight (J M times the material
    block), P = +1 on p / stresses and -1 on velocities.  It follows from
    exact summation by parts on affine elements and the symmetric,
    velocity/stress-decoupled upwind dissipation, and lets the adjoint run on
    the forward operator.  Absorbing faces keep it: their boundary term is
    -1/2 W |A_n|, and |A_n| couples velocities with velocities and stresses
    (pressure) with stresses only."""
    N = 2
    mesh = di.kuhn_box(2, 1, 1, jitter=0.15, seed=3)
    geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo)
    coef = di.acoustic_loguniform(mesh, 5) if physics == "acoustic" else di.elastic_loguniform(mesh, 5)
    mask = None
    if absorbing:  # every other unpaired face
        mask = geo.wall & (np.arange(geo.K * 4).reshape(geo.K, 4) % 2 == 0)
        assert 0 < mask.sum() < geo.wall.sum()
    o = make_oracle(physics, geo, coef, absorbing=mask)
    K, NF, Np = geo.K, o.nfields, geo.ref.Np
    n = K * NF * Np
    A = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        A[:, i] = o.rhs(e.reshape(K, NF, Np)).ravel()
    W = np.zeros((n, n))
    for k in range(K):
        if physics == "acoustic":
            rho, c = coef[k]
            C = np.diag([1 / (rho * c * c), rho, rho, rho])
            P = np.array([1, -1, -1, -1.0])
        else:
            rho, lam, mu = coef[k]
            C = np.zeros((9, 9))
            C[:3, :3] = rho * np.eye(3)
            t = np.array([1, 1, 1, 0, 0, 0.0])
            C[3:, 3:] = (np.diag([1, 1, 1, 2, 2, 2.0]) - lam / (3 * lam + 2 * mu) * np.outer(t, t)) / (2 * mu)
            P = np.array([-1, -1, -1, 1, 1, 1, 1, 1, 1.0])
        s = slice(k * NF * Np, (k + 1) * NF * Np)
        W[s, s] = np.kron(C, geo.J[k] * geo.ref.M)
    Pm = np.kron(np.eye(K), np.kron(np.diag(P), np.eye(Np)))
    rhs = Pm @ W @ A @ Pm @ np.linalg.inv(W)
    assert np.abs(A.T - rhs).max() <= 1e-11 * np.abs(A).max()
    # and the energy is dissipated: W A + A^T W is negative semidefinite
    S = W @ A
    assert np.linalg.eigvalsh(S + S.T).max() <= 1e-12 * np.abs(S).max()
