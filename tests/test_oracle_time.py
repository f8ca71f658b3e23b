"""Pins of the oracle's time integration and of the whole scheme (no GPU).

* AB3 (eq. (4)) on y' = lam y against the closed-form solution of the
  recurrence (roots of its characteristic cubic), plus observed order 3.
* The time-step recipe keeps dt * spec(L) inside the AB3 stability region
  (eigenvalues of the assembled operator on small meshes).
* Fully discrete energy is non-increasing over 100 steps (upwind flux).
* Plane waves on periodic boxes and the rigid-box standing mode converge at
  rate >= N + 1 - 0.3 against the exact solutions of the PDEs.
"""

import math

import numpy as np
import pytest

import dginputs as di
from oracle.dg import AB3Stepper, AcousticOracle, ElasticOracle, ab3_coefficients
from oracle.mesh import build_mesh


class _Scalar:
    def __init__(self, lam):
        self.lam = lam

    def rhs(self, q):
        return self.lam * q


def test_ab3_matches_closed_form_recurrence():
    lam, h, y0 = -0.7 + 0.3j, 0.05, 1.0 + 0.0j
    st = AB3Stepper(_Scalar(lam), np.array([y0]))
    z = h * lam
    ys = [y0]
    for _ in range(40):
        ys.append(st.step(1, h)[0])
    # start-up values: forward Euler, then the two-step formula
    y1 = y0 * (1 + z)
    y2 = y1 + z * (1.5 * y1 - 0.5 * y0)
    assert abs(ys[1] - y1) < 1e-15 and abs(ys[2] - y2) < 1e-15
    # from m = 2 on: y_m = sum_i c_i x_i^(m-2) with the roots of
    # x^3 - x^2 - z (23 x^2 - 16 x + 5) / 12 = 0, fixed by y_2, y_3, y_4
    roots = np.roots([1.0, -1.0 - 23.0 * z / 12.0, 16.0 * z / 12.0, -5.0 * z / 12.0])
    y3 = y2 + z * (23 * y2 - 16 * y1 + 5 * y0) / 12
    Vm = np.array([[1, 1, 1], roots, roots**2])
    c = np.linalg.solve(Vm, np.array([y0, y1, y2]))
    # the recurrence holds from m=3 with y0,y1,y2 as its initial values
    for m in range(3, 41):
        closed = np.sum(c * roots**m)
        assert abs(ys[m] - closed) < 1e-12 * max(1.0, abs(closed))
    assert abs(ys[3] - y3) < 1e-15
    assert ab3_coefficients(5) == (23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0)


def test_ab3_third_order():
    lam, T = -1.3, 1.0
    errs = []
    for ns in (20, 40, 80):
        h = T / ns
        hist = (np.array([lam * math.exp(-lam * h)]), np.array([lam * math.exp(-2 * lam * h)]))
        st = AB3Stepper(_Scalar(lam), np.array([1.0]), history=hist, step_index=2)
        errs.append(abs(st.step(ns, h)[0] - math.exp(lam * T)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.9)


def _assemble(o, K, nf, Np):
    n = K * nf * Np
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = o.rhs(e.reshape(K, nf, Np)).ravel()
    return A


@pytest.mark.parametrize(
    "physics,N,n",
    [("acoustic", 1, 2), ("acoustic", 2, 2), ("acoustic", 4, 1), ("elastic", 1, 2), ("elastic", 3, 1)],
)
def test_time_step_recipe_is_ab3_stable(physics, N, n):
    m = di.kuhn_box(n, jitter=0.1 if n > 1 else 0.0, seed=3)
    geo = build_mesh(N, m.elem_xyz, m.elem_topo, None)
    if physics == "acoustic":
        coef = di.acoustic_two_layer(m)
        o, nf = AcousticOracle(geo, coef), 4
    else:
        coef = di.elastic_loguniform(m, 1)
        o, nf = ElasticOracle(geo, coef), 9
    lam = np.linalg.eigvals(_assemble(o, geo.K, nf, geo.ref.Np))
    assert lam.real.max() < 1e-10  # upwind DG: no growing mode
    dt = di.time_step(m, N, di.max_wave_speed(coef, physics))
    worst = 0.0
    for zz in dt * lam:
        r = np.roots([1.0, -1.0 - 23.0 * zz / 12.0, 16.0 * zz / 12.0, -5.0 * zz / 12.0])
        worst = max(worst, np.abs(r).max())
    assert worst <= 1.0 + 1e-9


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_discrete_energy_non_increasing(physics):
    """After the forward-Euler start the energy never grows.

    The start step itself changes the quadratic energy by exactly
    dt <q, r>_E + dt^2/2 <r, r>_E (Euler is not energy stable: the second
    term is positive); from then on AB3 with the upwind flux decreases it.
    """
    m = di.kuhn_box(3, jitter=0.1, seed=0)
    N = 2
    geo = build_mesh(N, m.elem_xyz, m.elem_topo, None)
    if physics == "acoustic":
        coef = di.acoustic_two_layer(m)
        o = AcousticOracle(geo, coef)
        q0 = np.moveaxis(di.acoustic_gaussian(geo.xyz), 0, 1)
    else:
        coef = di.elastic_loguniform(m, 1)
        o = ElasticOracle(geo, coef)
        q0 = np.moveaxis(di.elastic_gaussian(geo.xyz), 0, 1)
    dt = di.time_step(m, N, di.max_wave_speed(coef, physics))
    st = AB3Stepper(o, q0)
    E = [o.energy(st.q)]
    for _ in range(100):
        st.step(1, dt)
        E.append(o.energy(st.q))
    E = np.array(E)
    r0 = o.rhs(q0)
    predicted = E[0] + dt * o.energy_rate(q0) + dt * dt * o.energy(r0)
    assert abs(E[1] - predicted) <= 1e-12 * E[0]
    assert np.all(E[2:] <= E[1:-1] * (1.0 + 1e-12))
    assert E[-1] < E[0]


def _plane_wave_error(physics, N, n, kind="P", T=0.1):
    m = di.kuhn_box(n, periodic=True)
    geo = build_mesh(N, m.elem_xyz, m.elem_topo, m.period)
    if physics == "acoustic":
        o = AcousticOracle(geo, di.acoustic_constant(m))
        mv, c = (1, 1, 0), 1.0

        def exact(t):
            return np.moveaxis(di.acoustic_plane_wave(geo.xyz, mv, t=t), 0, 1)
    else:
        o = ElasticOracle(geo, di.elastic_constant(m, 1.0, 1.0, 1.0))
        mv, c = (1, 0, 1), math.sqrt(3.0)

        def exact(t):
            return np.moveaxis(di.elastic_plane_wave(geo.xyz, mv, kind=kind, t=t), 0, 1)
    ns = int(math.ceil(T / di.time_step(m, N, c)))
    dt = T / ns
    # exact-history start-up so that the scheme is third order from step 0
    st = AB3Stepper(o, exact(0.0), history=(o.rhs(exact(-dt)), o.rhs(exact(-2 * dt))), step_index=2)
    st.step(ns, dt)
    return o.rel_l2(st.q, exact(T))[0]


@pytest.mark.parametrize(
    "physics,kind,N,meshes",
    [
        ("acoustic", "P", 1, (8, 16)),
        ("acoustic", "P", 2, (6, 12)),
        ("acoustic", "P", 3, (4, 8)),
        ("acoustic", "P", 4, (3, 6)),
        ("elastic", "P", 2, (4, 8)),
        ("elastic", "S", 3, (3, 6)),
    ],
)
def test_plane_wave_convergence(physics, kind, N, meshes):
    e = [_plane_wave_error(physics, N, n, kind) for n in meshes]
    rate = math.log(e[0] / e[1]) / math.log(meshes[1] / meshes[0])
    assert rate >= N + 1 - 0.3, (e, rate)


def test_rigid_box_standing_mode_converges():
    # p = cos(pi x) cos(pi y) cos(pi z) cos(sqrt(3) pi t), rho = c = 1,
    # v = -grad(cos pi x cos pi y cos pi z) sin(sqrt3 pi t) / (sqrt3 pi)
    N, T = 2, 0.1
    w = math.sqrt(3.0) * math.pi

    def exact(x, t):
        cx, cy, cz = (np.cos(math.pi * x[..., i]) for i in range(3))
        sx, sy, sz = (np.sin(math.pi * x[..., i]) for i in range(3))
        out = np.zeros((4,) + x.shape[:-1])
        out[0] = cx * cy * cz * math.cos(w * t)
        s = math.sin(w * t) * math.pi / w
        out[1] = sx * cy * cz * s
        out[2] = cx * sy * cz * s
        out[3] = cx * cy * sz * s
        return np.moveaxis(out, 0, 1)

    errs = []
    for n in (3, 6):
        m = di.kuhn_box(n)
        geo = build_mesh(N, m.elem_xyz, m.elem_topo, None)
        o = AcousticOracle(geo, di.acoustic_constant(m))
        ns = int(math.ceil(T / di.time_step(m, N, 1.0)))
        dt = T / ns
        st = AB3Stepper(o, exact(geo.xyz, 0.0), history=(o.rhs(exact(geo.xyz, -dt)), o.rhs(exact(geo.xyz, -2 * dt))), step_index=2)
        st.step(ns, dt)
        errs.append(o.rel_l2(st.q, exact(geo.xyz, T))[0])
    assert math.log2(errs[0] / errs[1]) >= N + 1 - 0.3, errs
