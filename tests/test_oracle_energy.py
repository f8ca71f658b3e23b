"""Absolute normalisation of the oracle's discrete energy (no GPU).

For fields that are polynomials of degree <= N in the physical coordinates,
the nodal interpolant is exact and the mass matrix integrates their products
exactly, so the discrete energy must equal the continuous energy of the
state, integrated here by a collapsed Gauss-Legendre cubature over each
physical tetrahedron (Duffy map of the unit simplex, volume from the vertex
determinant; nothing from the oracle's geometry or reference element):

  acoustic  1/2 int p^2/(rho c^2) + rho |v|^2 dx   (potential + kinetic);
  elastic   1/2 int rho |v|^2 + sigma : eps dx, with eps the strain that
            Hooke's law sigma = lambda tr(eps) I + 2 mu eps maps to sigma,
            obtained by inverting the 6x6 Voigt stiffness numerically.

A missing 1/2, a wrong compliance term or a wrong element volume factor in
the oracle's energy would fail here; the energy-rate tests cannot see an
overall factor.
"""

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

import dginputs as di
from oracle.dg import make_oracle
from oracle.mesh import build_mesh


def _simplex_rule(q):
    """Points (xi, eta, zeta) and weights on the unit simplex, exact for
    polynomials of degree <= 2q - 3."""
    x, w = leggauss(q)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    u, v, t = np.meshgrid(x, x, x, indexing="ij")
    wu, wv, wt = np.meshgrid(w, w, w, indexing="ij")
    xi = u
    eta = v * (1.0 - u)
    zeta = t * (1.0 - u) * (1.0 - v)
    W = wu * wv * wt * (1.0 - u) ** 2 * (1.0 - v)
    return np.stack([xi.ravel(), eta.ravel(), zeta.ravel()], 1), W.ravel()


def _poly_fields(nf, N, rng):
    mons = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]
    coef = rng.standard_normal((nf, len(mons)))

    def f(x):
        return np.stack([sum(cf * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c
                             for cf, (a, b, c) in zip(coef[i], mons)) for i in range(nf)])

    return f


def _voigt_compliance(lam, mu):
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] = lam + 2.0 * mu
    C[np.arange(3, 6), np.arange(3, 6)] = mu
    return np.linalg.inv(C)


def _continuous_energy(physics, mesh, coef, f, N):
    pts, W = _simplex_rule(N + 3)
    total = 0.0
    for k in range(mesh.K):
        x = mesh.elem_xyz[k]
        E = np.stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]], axis=1)
        vol = abs(np.linalg.det(E))
        X = x[0] + pts @ E.T
        u = f(X)  # (nf, npts)
        if physics == "acoustic":
            rho, c = coef[k]
            dens = u[0] ** 2 / (rho * c * c) + rho * np.sum(u[1:4] ** 2, axis=0)
        else:
            rho, lam, mu = coef[k]
            S = _voigt_compliance(lam, mu)
            sig = u[3:9]  # (xx, yy, zz, yz, xz, xy); Voigt strain = S sig
            dens = rho * np.sum(u[0:3] ** 2, axis=0) + np.einsum("ip,ij,jp->p", sig, S, sig)
        total += 0.5 * vol * np.dot(W, dens)
    return total


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("N", [1, 2, 4, 6])
def test_energy_equals_continuous_energy_of_polynomial_state(physics, N):
    rng = np.random.default_rng(100 + N)
    mesh = di.kuhn_box(2, jitter=0.1, seed=N)
    geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo)
    coef = di.acoustic_loguniform(mesh, 5) if physics == "acoustic" else di.elastic_loguniform(mesh, 5)
    nf = 4 if physics == "acoustic" else 9
    f = _poly_fields(nf, N, rng)
    q = np.moveaxis(f(geo.xyz), 0, 1)  # (K, nf, Np)
    e_disc = make_oracle(physics, geo, coef).energy(q)
    e_cont = _continuous_energy(physics, mesh, coef, f, N)
    assert e_cont > 0.0
    assert abs(e_disc - e_cont) <= 1e-11 * e_cont


def test_simplex_rule_volume_and_moments():
    pts, W = _simplex_rule(5)
    assert abs(W.sum() - 1.0 / 6.0) < 1e-15
    # int xi^a eta^b zeta^c over the unit simplex = a! b! c! / (a + b + c + 3)!
    from math import factorial

    for a, b, c in [(1, 0, 0), (2, 1, 0), (1, 1, 1), (3, 2, 2)]:
        exact = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
        got = np.dot(W, pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c)
        assert abs(got - exact) < 1e-15
