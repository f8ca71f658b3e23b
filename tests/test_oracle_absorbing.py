"""Pins of the oracle's absorbing boundary faces (no GPU).

Absorbing faces take a zero exterior state with the element's own
coefficients, so that the upwind flux of Sec. 2.1 lets no characteristic in
(a reading: Sec. 5 lists artificial boundary conditions as future work).
The pins rest on the PDE and its characteristics, not on the oracle:

* An outgoing polynomial plane wave (degree <= N, P-, S- or acoustic, on a
  box that is periodic across the wave and absorbing at its two ends, the
  profile vanishing on the inflow end) carries no incoming characteristic
  at either end, so r equals the exact PDE right-hand side at every node.
  With reflecting walls at the ends the same state is not steady-exact: the
  pin tells the two boundary kinds apart.
* For a continuous polynomial state every interior jump vanishes, and the
  semi-discrete energy rate reduces to the boundary terms.  Splitting the
  face state into characteristics gives, per absorbing face,
      acoustic  -1/2 int (p^2/Z + Z v_n^2) dS,
      elastic   -1/2 int (s_nn^2/Z_p + Z_p v_n^2 + |t_t|^2/Z_s + Z_s |v_t|^2) dS
  (t = s n, t_t and v_t the tangential parts), integrated here by a
  collapsed Gauss rule over the physical faces.
* The energy rate is <= 0 for random states and random coefficients.
* A normally incident pulse leaves the box: after it has crossed the
  outflow face, less than 1e-6 of its energy remains (measured 1.1e-8 at
  N = 3; a rigid wall keeps all of it).
"""

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

import dginputs as di
from oracle.dg import VOIGT, AB3Stepper, make_oracle
from oracle.mesh import build_mesh


def _slab(N, nx=4, ny=3, nz=3, jitter=0.1, seed=3):
    """Box open along x (absorbing or walls at x = 0, 1), periodic in y, z
    (periodic identification through vertex ids needs three subcubes or more
    per periodic direction)."""
    m = di.kuhn_box(nx, ny, nz, jitter=jitter, seed=seed, periodic=(False, True, True))
    geo = build_mesh(N, m.elem_xyz, m.elem_topo, m.period)
    return m, geo


def _poly(x, N, rng):
    """x * Q(x) with Q a random polynomial of degree N - 1 (zero at x = 0)."""
    c = rng.standard_normal(N)
    val = sum(ci * x ** (i + 1) for i, ci in enumerate(c))
    der = sum((i + 1) * ci * x**i for i, ci in enumerate(c))
    return val, der


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_acoustic_outgoing_wave_is_exact(N):
    m, geo = _slab(N)
    rho, c = 1.3, 0.8
    Z = rho * c
    coef = np.tile([rho, c], (geo.K, 1))
    assert geo.wall.sum() == 2 * 2 * 3 * 3  # the two x planes, 18 faces each
    X = geo.xyz[..., 0]
    f, df = _poly(X, N, np.random.default_rng(N))
    q = np.zeros((geo.K, 4, geo.ref.Np))
    q[:, 0] = f
    q[:, 1] = f / Z  # right-going: p = Z v_x
    exact = np.zeros_like(q)
    exact[:, 0] = -c * df  # -rho c^2 d(v_x)/dx
    exact[:, 1] = -df / rho
    r = make_oracle("acoustic", geo, coef, absorbing=geo.wall).rhs(q)
    np.testing.assert_allclose(r, exact, atol=1e-9 * (1 + np.abs(exact).max()))
    # the same state against rigid walls is not exact at the outflow end
    r_wall = make_oracle("acoustic", geo, coef).rhs(q)
    assert np.abs(r_wall - exact).max() > 1e-3 * np.abs(exact).max()


@pytest.mark.parametrize("kind", ["P", "S"])
@pytest.mark.parametrize("N", [1, 2, 4])
def test_elastic_outgoing_wave_is_exact(kind, N):
    m, geo = _slab(N)
    rho, lam, mu = 1.2, 0.9, 0.7
    cp, cs = np.sqrt((lam + 2 * mu) / rho), np.sqrt(mu / rho)
    coef = np.tile([rho, lam, mu], (geo.K, 1))
    X = geo.xyz[..., 0]
    f, df = _poly(X, N, np.random.default_rng(10 + N))
    q = np.zeros((geo.K, 9, geo.ref.Np))
    exact = np.zeros_like(q)
    if kind == "P":  # v = f x, s = -(lam I + 2 mu x x^T) f / cp
        q[:, 0] = f
        q[:, 3] = -(lam + 2 * mu) * f / cp
        q[:, 4] = -lam * f / cp
        q[:, 5] = -lam * f / cp
        exact[:, 0] = -(lam + 2 * mu) * df / (cp * rho)  # (1/rho) d s_xx / dx
        exact[:, 3] = (lam + 2 * mu) * df  # lam div v + 2 mu dv_x/dx
        exact[:, 4] = lam * df
        exact[:, 5] = lam * df
    else:  # v = f y, s_xy = -mu f / cs
        q[:, 1] = f
        q[:, 8] = -mu * f / cs
        exact[:, 1] = -mu * df / (cs * rho)  # (1/rho) d s_xy / dx
        exact[:, 8] = mu * df  # mu (dv_y/dx + dv_x/dy)
    r = make_oracle("elastic", geo, coef, absorbing=geo.wall).rhs(q)
    np.testing.assert_allclose(r, exact, atol=1e-9 * (1 + np.abs(exact).max()))
    r_wall = make_oracle("elastic", geo, coef).rhs(q)
    assert np.abs(r_wall - exact).max() > 1e-3 * np.abs(exact).max()


def _triangle_rule(q):
    """Points (a, b) and weights on the unit triangle (Duffy-collapsed Gauss),
    exact for degree <= 2q - 2."""
    x, w = leggauss(q)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    u, v = np.meshgrid(x, x, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    return np.stack([u.ravel(), (v * (1.0 - u)).ravel()], 1), (wu * wv * (1.0 - u)).ravel()


def _boundary_rate(physics, mesh, geo, coef, f, N):
    """-1/2 sum over unpaired faces of the characteristic dissipation."""
    pts, W = _triangle_rule(N + 2)
    total = 0.0
    xyz = mesh.elem_xyz
    for k, fc in zip(*np.nonzero(geo.wall)):
        # the vertex triple whose outward normal (away from the fourth
        # vertex) is the wall's: that is the face
        best, tri = -2.0, None
        for opp in range(4):
            t3 = xyz[k, [v for v in range(4) if v != opp]]
            nrm = np.cross(t3[1] - t3[0], t3[2] - t3[0])
            nrm = nrm / np.linalg.norm(nrm)
            if np.dot(nrm, xyz[k, opp] - t3[0]) > 0:
                nrm = -nrm
            d = np.dot(nrm, geo.normals[k, fc])
            if d > best:
                best, tri = d, t3
        assert best > 1.0 - 1e-12
        e1, e2 = tri[1] - tri[0], tri[2] - tri[0]
        area2 = np.linalg.norm(np.cross(e1, e2))
        n = geo.normals[k, fc]
        X = tri[0] + pts[:, :1] * e1 + pts[:, 1:] * e2
        u = f(X)  # (nf, npts)
        if physics == "acoustic":
            rho, c = coef[k]
            Z = rho * c
            p, vn = u[0], n @ u[1:4]
            dens = p**2 / Z + Z * vn**2
        else:
            rho, lam, mu = coef[k]
            Zp, Zs = np.sqrt(rho * (lam + 2 * mu)), np.sqrt(rho * mu)
            S = np.zeros((3, 3, u.shape[1]))
            for a, (i, j) in enumerate(VOIGT):
                S[i, j] = S[j, i] = u[3 + a]
            t = np.einsum("ijp,j->ip", S, n)
            v = u[0:3]
            snn, vn = n @ t, n @ v
            tt, vt = t - snn * n[:, None], v - vn * n[:, None]
            dens = snn**2 / Zp + Zp * vn**2 + np.sum(tt**2, 0) / Zs + Zs * np.sum(vt**2, 0)
        total += -0.5 * area2 * np.dot(W, dens)
    return total


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_energy_rate_of_polynomial_state_is_the_boundary_dissipation(physics, N):
    mesh = di.kuhn_box(2, jitter=0.1, seed=20 + N)
    geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo)
    coef = (di.acoustic_constant(mesh, 1.4, 0.9) if physics == "acoustic"
            else di.elastic_constant(mesh, 1.1, 0.8, 0.6))
    nf = 4 if physics == "acoustic" else 9
    rng = np.random.default_rng(30 + N)
    mons = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]
    cf = rng.standard_normal((nf, len(mons)))

    def f(x):
        return np.stack([sum(w * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c
                             for w, (a, b, c) in zip(cf[i], mons)) for i in range(nf)])

    q = np.moveaxis(f(geo.xyz), 0, 1)
    rate = make_oracle(physics, geo, coef, absorbing=geo.wall).energy_rate(q)
    ref = _boundary_rate(physics, mesh, geo, coef, f, N)
    assert ref < 0.0
    assert abs(rate - ref) <= 1e-10 * abs(ref)


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_energy_rate_nonpositive_random(physics):
    mesh = di.kuhn_box(2, jitter=0.1, seed=5)
    geo = build_mesh(3, mesh.elem_xyz, mesh.elem_topo)
    coef = di.acoustic_loguniform(mesh, 6) if physics == "acoustic" else di.elastic_loguniform(mesh, 6)
    rng = np.random.default_rng(8)
    absorbing = geo.wall & (rng.random(geo.wall.shape) < 0.5)
    assert 0 < absorbing.sum() < geo.wall.sum()
    o = make_oracle(physics, geo, coef, absorbing=absorbing)
    for _ in range(5):
        q = rng.standard_normal((geo.K, o.nfields, geo.ref.Np))
        scale = o.energy(q)
        assert o.energy_rate(q) <= 1e-12 * scale


def test_absorbing_mask_must_be_unpaired_faces():
    mesh = di.kuhn_box(2, jitter=0.0)
    geo = build_mesh(1, mesh.elem_xyz, mesh.elem_topo)
    bad = geo.wall.copy()
    bad[np.nonzero(~geo.wall)[0][0], np.nonzero(~geo.wall)[1][0]] = True
    with pytest.raises(ValueError):
        make_oracle("acoustic", geo, di.acoustic_constant(mesh), absorbing=bad)


@pytest.mark.parametrize("absorb", [True, False])
def test_normally_incident_pulse_leaves_the_box(absorb):
    N = 3
    m, geo = _slab(N, nx=10, jitter=0.0)
    coef = np.tile([1.0, 1.0], (geo.K, 1))
    X = geo.xyz[..., 0]
    g = np.exp(-((X - 0.5) ** 2) / (2 * 0.08**2))
    q0 = np.zeros((geo.K, 4, geo.ref.Np))
    q0[:, 0] = g
    q0[:, 1] = g  # right-going
    o = make_oracle("acoustic", geo, coef, absorbing=geo.wall if absorb else None)
    dt = di.time_step(m, N, 1.0)
    nsteps = int(np.ceil(1.0 / dt))  # the pulse travels one box length
    e0 = o.energy(q0)
    q = AB3Stepper(o, q0).step(nsteps, dt)
    left = o.energy(q) / e0
    if absorb:
        assert left < 1e-6, left
    else:
        assert left > 0.9, left
