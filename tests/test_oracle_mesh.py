"""Pins of the oracle's geometry and connectivity (no GPU).

Checked against mesh facts computed another way: the box volume, physical
face areas from vertex cross products, the closed-surface identity
sum_f A_f n_f = 0, the Kuhn boundary-face count, exact physical gradients of
linear and degree-N fields, and coordinate agreement of paired face nodes.
"""

import numpy as np
import pytest

import dginputs as di
from oracle.mesh import build_mesh
from oracle.refelem import FACE_VERTS


@pytest.mark.parametrize("periodic", [False, True])
def test_volumes_areas_normals(periodic):
    m = di.kuhn_box(3, 3, 4, lengths=(1.0, 1.0, 1.5), jitter=0.1, seed=5, periodic=periodic)
    geo = build_mesh(2, m.elem_xyz, m.elem_topo, m.period)
    assert np.all(geo.J > 0)
    assert abs(np.sum(4.0 / 3.0 * geo.J) - 1.5) < 1e-12
    x = m.elem_xyz
    area = np.stack(
        [0.5 * np.linalg.norm(np.cross(x[:, b] - x[:, a], x[:, c] - x[:, a]), axis=1) for a, b, c in FACE_VERTS],
        1,
    )
    # physical area = (area 2 of the parameter triangle) * sJ, sJ = Fscale * J
    np.testing.assert_allclose(2.0 * geo.Fscale * geo.J[:, None], area, rtol=1e-12)
    closed = np.einsum("kf,kfi->ki", area, geo.normals)
    np.testing.assert_allclose(closed, 0.0, atol=1e-13)
    # outward: the normal points away from the opposite vertex
    for f, (a, b, c) in enumerate(FACE_VERTS):
        d = ({0, 1, 2, 3} - {a, b, c}).pop()
        assert np.all(np.einsum("ki,ki->k", x[:, a] - x[:, d], geo.normals[:, f]) > 0)
    paired = ~geo.wall
    k, f = np.nonzero(paired)
    np.testing.assert_allclose(geo.normals[k, f], -geo.normals[geo.EToE[k, f], geo.EToF[k, f]], atol=1e-12)


@pytest.mark.parametrize("n", [2, 3])
def test_wall_face_count_and_pairing(n):
    m = di.kuhn_box(n, jitter=0.1, seed=1)
    geo = build_mesh(3, m.elem_xyz, m.elem_topo, None)
    assert geo.wall.sum() == 6 * 2 * n * n
    k, f = np.nonzero(~geo.wall)
    k2, f2 = geo.EToE[k, f], geo.EToF[k, f]
    assert np.all(geo.EToE[k2, f2] == k) and np.all(geo.EToF[k2, f2] == f)
    xf = geo.xyz[:, geo.ref.Fmask]  # (K, 4, Nfp, 3)
    own = xf[k, f]
    nb = xf[k2, f2][np.arange(len(k))[:, None], geo.nbr_node[k, f]]
    np.testing.assert_allclose(own, nb, atol=1e-13)
    # the node map is an involution
    back = geo.nbr_node[k2, f2][np.arange(len(k))[:, None], geo.nbr_node[k, f]]
    assert np.all(back == np.arange(geo.ref.Nfp)[None, :])


def test_periodic_pairing_has_no_walls():
    m = di.kuhn_box(3, periodic=True, jitter=0.05, seed=2)
    geo = build_mesh(2, m.elem_xyz, m.elem_topo, m.period)
    assert not geo.wall.any()
    k, f = np.nonzero(~geo.wall)
    xf = geo.xyz[:, geo.ref.Fmask]
    d = xf[k, f] - xf[geo.EToE[k, f], geo.EToF[k, f]][np.arange(len(k))[:, None], geo.nbr_node[k, f]]
    d -= np.round(d)
    np.testing.assert_allclose(d, 0.0, atol=1e-13)


@pytest.mark.parametrize("N", [1, 3, 5])
def test_physical_gradient_exact_for_polynomials(N):
    m = di.kuhn_box(2, jitter=0.1, seed=9)
    geo = build_mesh(N, m.elem_xyz, m.elem_topo, None)
    X, Y, Z = geo.xyz[..., 0], geo.xyz[..., 1], geo.xyz[..., 2]
    # a degree-N polynomial in the physical coordinates
    u = X**N + 2.0 * Y ** (N - 1) * Z + 0.5 * X * Y ** (N - 1)
    du = [
        N * X ** (N - 1) + 0.5 * Y ** (N - 1),
        (N - 1) * (2.0 * Y ** max(N - 2, 0) * Z + 0.5 * X * Y ** max(N - 2, 0)),
        2.0 * Y ** (N - 1),
    ]
    Du = np.stack([u @ geo.ref.D[j].T for j in range(3)], 1)
    grad = np.einsum("kij,kjn->kin", geo.G, Du)
    for i in range(3):
        np.testing.assert_allclose(grad[:, i], du[i], atol=1e-10)


@pytest.mark.parametrize("periodic", [False, True])
def test_relabelled_vertices_pair_faces_in_all_six_orientations(periodic):
    """Random even vertex orders per element make shared faces meet under all
    six relative orientations; paired face nodes still coincide in space."""
    m = di.relabel_vertices(di.kuhn_box(3, periodic=periodic, jitter=0.05, seed=5), seed=11)
    dets = np.linalg.det(np.stack([m.elem_xyz[:, i] - m.elem_xyz[:, 0] for i in (1, 2, 3)], axis=-1))
    assert np.all(dets > 0.0)
    for N in (1, 3, 4):
        geo = build_mesh(N, m.elem_xyz, m.elem_topo, m.period)
        k, f = np.nonzero(~geo.wall)
        patterns = {tuple(r) for r in geo.nbr_node[k, f]}
        assert len(patterns) == 6
        xf = geo.xyz[:, geo.ref.Fmask]
        d = xf[k, f] - xf[geo.EToE[k, f], geo.EToF[k, f]][np.arange(len(k))[:, None], geo.nbr_node[k, f]]
        if periodic:
            d -= np.round(d)
        np.testing.assert_allclose(d, 0.0, atol=1e-13)
