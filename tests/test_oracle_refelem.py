"""Pins of the oracle's reference tetrahedron against closed forms, textbook
values and an independent cubature (no GPU).

Each check uses something other than the oracle itself: the node counts the
paper prints in Table 4, the P1 mass matrix and derivative matrices written
out by hand, exact derivatives of monomials, the Gauss-Lobatto points from
SciPy's Gauss-Jacobi routine, and integrals from a conical-product Gauss
cubature.
"""

import itertools
import math
import os

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy.special import roots_jacobi

from oracle.refelem import (
    FACE_VERTS,
    REF_VERTS,
    face_param_coords,
    n_face_nodes,
    n_nodes,
    reference_element,
)

DEGREES = list(range(1, 9))
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table4_node_counts.txt")


def test_node_counts_match_table4():
    rows = np.loadtxt(GOLDEN, dtype=int)
    for N, Np, Np3 in rows:
        assert n_nodes(N) == Np
        assert 3 * n_nodes(N) == Np3
        ref = reference_element(int(N))
        assert ref.r.shape == (Np, 3)
        assert ref.Fmask.shape == (4, (N + 1) * (N + 2) // 2)


def test_p1_closed_forms():
    ref = reference_element(1)
    np.testing.assert_allclose(ref.r, REF_VERTS, atol=1e-15)
    Dr = np.tile([-0.5, 0.5, 0.0, 0.0], (4, 1))
    Ds = np.tile([-0.5, 0.0, 0.5, 0.0], (4, 1))
    Dt = np.tile([-0.5, 0.0, 0.0, 0.5], (4, 1))
    np.testing.assert_allclose(ref.D[0], Dr, atol=1e-14)
    np.testing.assert_allclose(ref.D[1], Ds, atol=1e-14)
    np.testing.assert_allclose(ref.D[2], Dt, atol=1e-14)
    # textbook P1 mass matrix on a tetrahedron of volume 4/3: V/20 (1 + delta)
    M = (4.0 / 3.0) / 20.0 * (np.ones((4, 4)) + np.eye(4))
    np.testing.assert_allclose(ref.M, M, atol=1e-14)


def _monomials(N):
    return [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]


@pytest.mark.parametrize("N", DEGREES)
def test_exact_differentiation_of_monomials(N):
    ref = reference_element(N)
    r, s, t = ref.r.T
    worst = 0.0
    for a, b, c in _monomials(N):
        u = r**a * s**b * t**c
        exact = [
            a * r ** max(a - 1, 0) * s**b * t**c,
            b * r**a * s ** max(b - 1, 0) * t**c,
            c * r**a * s**b * t ** max(c - 1, 0),
        ]
        for j in range(3):
            worst = max(worst, np.abs(ref.D[j] @ u - exact[j]).max())
    assert worst <= 1e-12
    np.testing.assert_allclose(ref.D.sum(axis=2), 0.0, atol=1e-12)


@pytest.mark.parametrize("N", DEGREES)
def test_edge_nodes_are_gauss_lobatto(N):
    ref = reference_element(N)
    lat = ref.lattice
    on_edge = (lat[:, 2] == 0) & (lat[:, 3] == 0)  # edge v1 -> v2, coordinate r
    r_edge = np.sort(ref.r[on_edge, 0])
    inner = np.sort(roots_jacobi(N - 1, 1.0, 1.0)[0]) if N > 1 else np.array([])
    expect = np.concatenate([[-1.0], inner, [1.0]])
    np.testing.assert_allclose(r_edge, expect, atol=1e-13)
    np.testing.assert_allclose(ref.r[on_edge, 1:], -1.0, atol=1e-14)


@pytest.mark.parametrize("N", DEGREES)
def test_node_set_symmetric_under_vertex_permutations(N):
    ref = reference_element(N)
    r, s, t = ref.r.T
    lam = np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], 1)
    index = {tuple(l): n for n, l in enumerate(ref.lattice)}
    for perm in itertools.permutations(range(4)):
        for n, l in enumerate(ref.lattice):
            m = index[tuple(l[list(perm)])]
            np.testing.assert_allclose(lam[m], lam[n][list(perm)], atol=1e-13)
    # the nodes of every face sit at the same parameter-triangle coordinates
    for f in range(4):
        np.testing.assert_allclose(face_param_coords(N, f), ref.face_xy, atol=1e-13)
    assert np.linalg.cond(ref.V) < 1e3


def _tet_cubature(q):
    x, w = leggauss(q)
    a, b, c = np.meshgrid(x, x, x, indexing="ij")
    wa, wb, wc = np.meshgrid(w, w, w, indexing="ij")
    r = (1 + a) * (1 - b) * (1 - c) / 4 - 1
    s = (1 + b) * (1 - c) / 2 - 1
    t = c
    W = wa * wb * wc * (1 - b) * (1 - c) ** 2 / 8
    return np.stack([r.ravel(), s.ravel(), t.ravel()], 1), W.ravel()


def _tri_cubature(q):
    x, w = leggauss(q)
    a, b = np.meshgrid(x, x, indexing="ij")
    wa, wb = np.meshgrid(w, w, indexing="ij")
    X = (1 + a) * (1 - b) / 2 - 1
    Y = b
    W = wa * wb * (1 - b) / 2
    return np.stack([X.ravel(), Y.ravel()], 1), W.ravel()


def _rand_poly(N, rng):
    mons = _monomials(N)
    coef = rng.standard_normal(len(mons))

    def f(p):
        return sum(cf * p[:, 0] ** a * p[:, 1] ** b * p[:, 2] ** c for cf, (a, b, c) in zip(coef, mons))

    return f


@pytest.mark.parametrize("N", DEGREES)
def test_mass_matrix_integrates_products_exactly(N):
    ref = reference_element(N)
    pts, W = _tet_cubature(N + 4)
    assert abs(W.sum() - 4.0 / 3.0) < 1e-14
    one = np.ones(ref.Np)
    assert abs(one @ ref.M @ one - 4.0 / 3.0) < 1e-12
    rng = np.random.default_rng(N)
    for _ in range(3):
        u, w = _rand_poly(N, rng), _rand_poly(N, rng)
        exact = np.sum(W * u(pts) * w(pts))
        disc = w(ref.r) @ ref.M @ u(ref.r)
        assert abs(disc - exact) <= 1e-11 * max(1.0, abs(exact))


@pytest.mark.parametrize("N", DEGREES)
def test_lift_reproduces_face_integrals(N):
    ref = reference_element(N)
    xy, W = _tri_cubature(N + 3)
    assert abs(W.sum() - 2.0) < 1e-14
    mu = np.stack([-(xy[:, 0] + xy[:, 1]) / 2, (1 + xy[:, 0]) / 2, (1 + xy[:, 1]) / 2], 1)
    rng = np.random.default_rng(100 + N)
    Nfp = ref.Nfp
    for f, (A, B, C) in enumerate(FACE_VERTS):
        P = mu @ REF_VERTS[[A, B, C]]  # cubature points on face f
        u, w = _rand_poly(N, rng), _rand_poly(N, rng)
        exact = np.sum(W * u(P) * w(P))
        uf = u(ref.r[ref.Fmask[f]])
        disc = w(ref.r) @ ref.M @ (ref.LIFT[:, f * Nfp : (f + 1) * Nfp] @ uf)
        assert abs(disc - exact) <= 1e-11 * max(1.0, abs(exact))


def test_face_mass_p1_closed_form():
    # linear triangle mass on T (area 2): A/12 (1 + delta)
    ref = reference_element(1)
    np.testing.assert_allclose(ref.Eface, (2.0 / 12.0) * (np.ones((3, 3)) + np.eye(3)), atol=1e-14)
    assert n_face_nodes(1) == 3 and math.isclose(ref.Eface.sum(), 2.0)
