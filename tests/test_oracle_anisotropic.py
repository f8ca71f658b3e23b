"""Pins of the oracle's anisotropic elastic right-hand side (no GPU).

The anisotropic medium (general 21-coefficient stiffness) is the paper's
future work (Sec. 5); the pins rest on the PDE, not on the oracle:

* with an isotropic stiffness the volume terms are those of the isotropic
  elastic oracle (Sec. 3.2), compared where every penalty vanishes: a
  continuous polynomial state, on the elements away from the walls;
* a continuous polynomial state of degree <= N in a homogeneous anisotropic
  medium gives the exact PDE right-hand side rho^-1 div s, C e(v) at the
  nodes of the elements away from the walls (no jumps there);
* the semi-discrete energy rate is <= 0 for random states in heterogeneous
  random media with walls and absorbing faces (the flux dissipates
  -(Z- Z+/(Z- + Z+)) |[v]|^2 - |[t]|^2/(Z- + Z+) per face, derived in the
  oracle's docstring);
* the discrete energy of a polynomial state equals its continuous energy
  1/2 int rho |v|^2 + s : C^-1 s (collapsed Gauss cubature);
* plane waves from the Christoffel eigenproblem converge at order >= N+1-0.3
  (periodic cube, exact-history AB3 start), as the isotropic ones do.
"""

import numpy as np
import pytest

import dginputs as di
from oracle.dg import AB3Stepper, AnisotropicElasticOracle, ElasticOracle, make_oracle, stiffness_matrix
from oracle.mesh import build_mesh


def _walled(n, N, seed=3):
    m = di.kuhn_box(n, jitter=0.1, seed=seed)
    geo = build_mesh(N, m.elem_xyz, m.elem_topo)
    return m, geo, ~geo.wall.any(axis=1)


def _poly_state(geo, N, rng):
    """Nine fields, each a random combination of x^a y^b z^c, a+b+c <= N,
    continuous across elements, and their exact gradients."""
    mons = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]
    cf = rng.standard_normal((9, len(mons)))
    X, Y, Z = (geo.xyz[..., i] for i in range(3))
    val = np.zeros((9,) + X.shape)
    grad = np.zeros((9, 3) + X.shape)
    for i in range(9):
        for w, (a, b, c) in zip(cf[i], mons):
            val[i] += w * X**a * Y**b * Z**c
            if a:
                grad[i, 0] += w * a * X ** (a - 1) * Y**b * Z**c
            if b:
                grad[i, 1] += w * b * X**a * Y ** (b - 1) * Z**c
            if c:
                grad[i, 2] += w * c * X**a * Y**b * Z ** (c - 1)
    return np.moveaxis(val, 0, 1), grad


def test_isotropic_stiffness_has_the_isotropic_volume_terms():
    N = 2
    m, geo, inner = _walled(3, N)
    assert inner.sum() > 0
    iso = np.tile([1.3, 0.8, 0.6], (geo.K, 1))
    q, _ = _poly_state(geo, N, np.random.default_rng(1))
    r_iso = ElasticOracle(geo, iso).rhs(q)[inner]
    r_an = AnisotropicElasticOracle(geo, di.anisotropic_from_isotropic(iso)).rhs(q)[inner]
    np.testing.assert_allclose(r_an, r_iso, atol=1e-9 * np.abs(r_iso).max())


@pytest.mark.parametrize("N", [1, 2, 3])
def test_polynomial_state_gives_the_pde_rhs(N):
    m, geo, inner = _walled(3, N, seed=5)
    row = di.anisotropic_random(di.kuhn_box(1), seed=7)[0]
    coef = np.tile(row, (geo.K, 1))
    rho, C = row[0], stiffness_matrix(row[1:])
    q, g = _poly_state(geo, N, np.random.default_rng(N))
    o = AnisotropicElasticOracle(geo, coef)
    r = o.rhs(q)
    # exact: rho^-1 sum_j d s_ij / d x_j and C e(v)
    vo = {(0, 0): 3, (1, 1): 4, (2, 2): 5, (1, 2): 6, (2, 1): 6, (0, 2): 7, (2, 0): 7, (0, 1): 8, (1, 0): 8}
    exact = np.zeros_like(q)
    for i in range(3):
        exact[:, i] = sum(g[vo[(i, j)], j] for j in range(3)) / rho
    e = np.stack([g[0, 0], g[1, 1], g[2, 2], g[1, 2] + g[2, 1], g[0, 2] + g[2, 0], g[0, 1] + g[1, 0]])
    exact[:, 3:9] = np.moveaxis(np.einsum("ab,bkn->akn", C, e), 0, 1)
    np.testing.assert_allclose(r[inner], exact[inner], atol=1e-9 * np.abs(exact).max())


@pytest.mark.parametrize("absorb", [False, True])
def test_energy_rate_nonpositive(absorb):
    m = di.kuhn_box(2, jitter=0.1, seed=9)
    geo = build_mesh(3, m.elem_xyz, m.elem_topo)
    coef = di.anisotropic_random(m, seed=11)
    mask = geo.wall & (np.random.default_rng(2).random(geo.wall.shape) < 0.5) if absorb else None
    o = make_oracle("anisotropic", geo, coef, absorbing=mask)
    rng = np.random.default_rng(4)
    for _ in range(4):
        q = rng.standard_normal((geo.K, 9, geo.ref.Np))
        assert o.energy_rate(q) <= 1e-12 * o.energy(q)


def test_energy_equals_continuous_energy():
    from numpy.polynomial.legendre import leggauss

    N = 2
    m = di.kuhn_box(2, jitter=0.1, seed=13)
    geo = build_mesh(N, m.elem_xyz, m.elem_topo)
    coef = di.anisotropic_random(m, seed=14)
    q, _ = _poly_state(geo, N, np.random.default_rng(15))
    e_disc = AnisotropicElasticOracle(geo, coef).energy(q)
    # continuous energy by a collapsed Gauss rule of the same polynomial
    rng = np.random.default_rng(15)
    mons = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]
    cf = rng.standard_normal((9, len(mons)))
    x, w = leggauss(N + 3)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    u, v, t = np.meshgrid(x, x, x, indexing="ij")
    wu, wv, wt = np.meshgrid(w, w, w, indexing="ij")
    pts = np.stack([u.ravel(), (v * (1 - u)).ravel(), (t * (1 - u) * (1 - v)).ravel()], 1)
    W = (wu * wv * wt * (1 - u) ** 2 * (1 - v)).ravel()
    total = 0.0
    for k in range(m.K):
        xv = m.elem_xyz[k]
        E = np.stack([xv[1] - xv[0], xv[2] - xv[0], xv[3] - xv[0]], axis=1)
        X = xv[0] + pts @ E.T
        f = np.stack([sum(wc * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c for wc, (a, b, c) in zip(cf[i], mons))
                      for i in range(9)])
        S = np.linalg.inv(stiffness_matrix(coef[k, 1:]))
        dens = coef[k, 0] * np.sum(f[0:3] ** 2, 0) + np.einsum("ap,ab,bp->p", f[3:9], S, f[3:9])
        total += 0.5 * abs(np.linalg.det(E)) * np.dot(W, dens)
    assert abs(e_disc - total) <= 1e-11 * total


@pytest.mark.parametrize("N,meshes", [(2, (4, 8)), (3, (3, 6))])
def test_plane_wave_convergence(N, meshes):
    """The fastest (quasi-P) plane wave along x in a random anisotropic
    medium, periodic box, one step of the time-step recipe, T = 0.1."""
    row = di.anisotropic_random(di.kuhn_box(1), seed=21)[0]
    errs = []
    for n in meshes:
        m = di.kuhn_box(n, periodic=True)
        geo = build_mesh(N, m.elem_xyz, m.elem_topo, m.period)
        coef = np.tile(row, (geo.K, 1))
        o = AnisotropicElasticOracle(geo, coef)

        def exact(t):
            return np.moveaxis(di.anisotropic_plane_wave(geo.xyz, (1, 0, 0), row[0], row[1:], mode=2, t=t), 0, 1)

        T = 0.1
        nsteps = int(np.ceil(T / di.time_step(m, N, di.max_wave_speed(coef, "anisotropic"))))
        dt = T / nsteps
        st = AB3Stepper(o, exact(0.0), history=(o.rhs(exact(-dt)), o.rhs(exact(-2 * dt))), step_index=2)
        errs.append(o.rel_l2(st.step(nsteps, dt), exact(T))[0])
    rate = np.log2(errs[0] / errs[1])
    assert rate >= N + 1 - 0.3, (errs, rate)
