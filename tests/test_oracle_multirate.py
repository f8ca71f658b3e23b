"""Pins of the oracle's two-rate Adams-Bashforth stepping (no GPU).

* The dense-output weights are the integrals of the Lagrange polynomial
  through the history: at a full step they are the weights of eq. (4)
  (23/12, -16/12, 5/12; the start-up's 1 and 3/2, -1/2), at half a step
  17/24, -7/24, 1/12 (5/8, -1/8; 1/2), and they integrate every polynomial
  of the history's degree exactly.
* With every element in one class the stepping is bit for bit the
  single-rate AB3 loop (all slow: steps of dt; all fast: twice as many of
  dt/2).
* On meshes with two classes (two wave-speed layers, and a mesh graded in
  size) the time-integration error, measured against single-rate AB3 with a
  64 times smaller step on the same semi-discretisation, falls at third
  order as dt halves (both runs started from the exact history).
* The discrete energy does not grow over the run after the start-up (AB3
  is not a contraction in general, so this is an observation on these
  cases, with a 1e-12 relative tolerance per step), while single-rate AB3
  at the macro step is unstable on the same mesh.
"""

from fractions import Fraction

import numpy as np
import pytest

import dginputs as di
from oracle.dg import AB3Stepper, make_oracle
from oracle.mesh import build_mesh
from oracle.multirate import TwoRateAB3, history_weights


def test_history_weights_full_step_are_the_ab_weights():
    assert history_weights(1, 1) == [Fraction(1)]
    assert history_weights(2, 1) == [Fraction(3, 2), Fraction(-1, 2)]
    assert history_weights(3, 1) == [Fraction(23, 12), Fraction(-16, 12), Fraction(5, 12)]


def test_history_weights_half_step():
    assert history_weights(1, Fraction(1, 2)) == [Fraction(1, 2)]
    assert history_weights(2, Fraction(1, 2)) == [Fraction(5, 8), Fraction(-1, 8)]
    assert history_weights(3, Fraction(1, 2)) == [Fraction(17, 24), Fraction(-7, 24), Fraction(1, 12)]


@pytest.mark.parametrize("theta", [Fraction(1, 3), Fraction(1, 2), Fraction(3, 4), Fraction(1)])
def test_history_weights_integrate_polynomials_exactly(theta):
    for deg in range(3):
        w = history_weights(deg + 1, theta)
        for p in range(deg + 1):  # f(s) = s^p
            approx = sum(wi * Fraction(-i) ** p for i, wi in enumerate(w))
            assert approx == theta ** (p + 1) / (p + 1)


def _two_layer_case(N=2, n=3, physics="acoustic"):
    m = di.kuhn_box(n, jitter=0.1, seed=11)
    geo = build_mesh(N, m.elem_xyz, m.elem_topo)
    cen = di.element_centroids(m)
    if physics == "acoustic":
        coef = np.where(cen[:, :1] < 0.5, [[1.0, 2.0]], [[1.0, 1.0]])  # c = 2 | 1
    else:
        coef = np.where(cen[:, :1] < 0.5, [[1.0, 2.0, 1.5]], [[1.0, 0.5, 0.375]])  # c_p = 2.35 | 1.17
    fast, dt = di.two_rate_classes(m, N, di.element_wave_speeds(coef, physics))
    q0 = np.ascontiguousarray(np.moveaxis(di.gaussian_pulses(geo.xyz, 4 if physics == "acoustic" else 9, sigma=0.15), 0, 1))
    return m, geo, coef, fast, dt, q0


@pytest.mark.parametrize("which", ["slow", "fast"])
def test_one_class_is_single_rate_ab3_bitwise(which):
    m, geo, coef, _, dt, q0 = _two_layer_case()
    o = make_oracle("acoustic", geo, coef)
    fast = np.full(geo.K, which == "fast")
    got = TwoRateAB3(o, q0, fast).macro_step(7, dt)
    ref = AB3Stepper(o, q0).step(7 if which == "slow" else 14, dt if which == "slow" else dt / 2)
    assert np.array_equal(got, ref)


def _past_rhs(o, q0, tau):
    """L q(-tau) of the semi-discrete solution q(t) = exp(t L) q0, from its
    Taylor series to third order (error O(tau^4), far below the O(dt^3)
    being measured): the exact history that a third-order start needs (an
    Euler / two-step start alone is second order)."""
    terms = [q0]
    for _ in range(3):
        terms.append(o.rhs(terms[-1]))
    q = sum((-tau) ** k / np.prod(np.arange(1, k + 1)) * t for k, t in enumerate(terms))
    return o.rhs(q)


def _temporal_rate(o, q0, fast, dt, T):
    n_ref = int(round(T / dt)) * 2 * 32
    d_ref = T / n_ref
    ref = AB3Stepper(o, q0, history=(_past_rhs(o, q0, d_ref), _past_rhs(o, q0, 2 * d_ref)), step_index=2)
    ref = ref.step(n_ref, d_ref)
    errs = []
    for k in range(3):
        d = dt / 2**k
        n = int(round(T / d))
        hist = ((_past_rhs(o, q0, d / 2), _past_rhs(o, q0, d)), (_past_rhs(o, q0, d), _past_rhs(o, q0, 2 * d)))
        q = TwoRateAB3(o, q0, fast, history=hist).macro_step(n, d)
        errs.append(o.rel_l2(q, ref)[0])
    return errs, [np.log2(errs[i] / errs[i + 1]) for i in range(2)]


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_third_order_on_two_speed_layers(physics):
    m, geo, coef, fast, dt, q0 = _two_layer_case(physics=physics)
    assert 0.3 < fast.mean() < 0.7  # both classes are large
    o = make_oracle(physics, geo, coef)
    errs, rates = _temporal_rate(o, q0, fast, dt, T=40 * dt)
    assert errs[0] > 1e-9  # the time error is well above rounding
    assert min(rates) >= 2.7, (errs, rates)


def test_third_order_on_graded_mesh():
    N = 2
    m = di.graded_kuhn_box(5, 2)  # cells 0.1 and 0.25 wide
    geo = build_mesh(N, m.elem_xyz, m.elem_topo)
    coef = np.tile([1.0, 1.0], (geo.K, 1))
    fast, dt = di.two_rate_classes(m, N, np.ones(geo.K))
    assert 0 < (~fast).sum() and 0 < fast.sum()
    q0 = np.ascontiguousarray(np.moveaxis(di.gaussian_pulses(geo.xyz, 4, sigma=0.2), 0, 1))
    o = make_oracle("acoustic", geo, coef)
    errs, rates = _temporal_rate(o, q0, fast, dt, T=40 * dt)
    assert errs[0] > 1e-9
    assert min(rates) >= 2.7, (errs, rates)


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_energy_does_not_grow(physics):
    """After the start-up (whose Euler step may raise the energy, as in the
    single-rate loop) the energy does not grow over 60 macro steps."""
    m, geo, coef, fast, dt, q0 = _two_layer_case(physics=physics)
    o = make_oracle(physics, geo, coef)
    st = TwoRateAB3(o, q0, fast)
    st.macro_step(1, dt)
    e_prev = e1 = o.energy(st.q)
    for _ in range(60):
        e = o.energy(st.macro_step(1, dt))
        assert e <= e_prev * (1 + 1e-12)
        e_prev = e
    assert e_prev < e1


def test_single_rate_at_the_macro_step_is_unstable_here():
    """The fast class needs its half step: single-rate AB3 at the macro step
    on the two-layer acoustic case grows the energy without bound, while
    the two-rate run above stays bounded."""
    m, geo, coef, fast, dt, q0 = _two_layer_case()
    o = make_oracle("acoustic", geo, coef)
    st = AB3Stepper(o, q0)
    e1 = o.energy(st.step(1, dt))
    e = o.energy(st.step(60, dt))
    assert e > 100 * e1
