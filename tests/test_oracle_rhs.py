"""Pins of the oracle's acoustic and elastic right-hand sides (no GPU).

* A constant state is steady (r = 0).
* A continuous degree-N polynomial state has zero penalty, so on elements
  away from walls r equals the exact PDE right-hand side at the nodes, with
  each element's own coefficients (also across material jumps).
* For a piecewise-constant state every face carries an exact Riemann
  problem; the test solves it from the characteristic relations of the PDE
  (written here independently of the paper's alpha / k notation) and checks
  that r is the lift of the strong-form correction n.(F(q*) - F(q^-)).
* The semi-discrete energy rate is <= 0 for random states.
"""

import numpy as np
import pytest

import dginputs as di
from oracle.dg import VOIGT, AcousticOracle, ElasticOracle
from oracle.mesh import build_mesh


def _mesh(n=3, periodic=False, N=2, jitter=0.1, seed=4):
    m = di.kuhn_box(n, periodic=periodic, jitter=jitter, seed=seed)
    return m, build_mesh(N, m.elem_xyz, m.elem_topo, m.period)


@pytest.mark.parametrize("periodic", [False, True])
def test_constant_state_is_steady(periodic):
    m, geo = _mesh(periodic=periodic)
    Np = geo.ref.Np
    ac = AcousticOracle(geo, di.acoustic_loguniform(m, 1))
    q = np.zeros((geo.K, 4, Np))
    q[:, 0] = 1.7
    assert np.abs(ac.rhs(q)).max() < 1e-12
    el = ElasticOracle(geo, di.elastic_loguniform(m, 2))
    q = np.zeros((geo.K, 9, Np))
    q[:, 0:3] = np.array([0.3, -1.1, 0.6])[:, None]
    assert np.abs(el.rhs(q)).max() < 1e-12
    if periodic:  # a uniform stress is steady only without traction-free walls
        q[:, 3:9] = np.array([1.0, 2.0, 3.0, 0.5, -0.4, 0.2])[:, None]
        assert np.abs(el.rhs(q)).max() < 1e-11


def _interior(geo):
    return ~geo.wall.any(axis=1)


@pytest.mark.parametrize("N", [1, 2, 4])
def test_acoustic_polynomial_state_matches_pde(N):
    m, geo = _mesh(n=3, N=N)
    coef = di.acoustic_loguniform(m, 7)
    ac = AcousticOracle(geo, coef)
    X, Y, Z = (geo.xyz[..., i] for i in range(3))
    # degree-N fields and their exact derivatives
    p = X ** (N - 1) * Y + Z
    u = Y**N - X * Z ** (N - 1)
    v = Z**N + X
    w = X * Y * Z ** (N - 2) if N >= 2 else X + Y
    q = np.stack([p, u, v, w], 1)
    dp = [(N - 1) * X ** max(N - 2, 0) * Y, X ** (N - 1), np.ones_like(Z)]
    div = -(Z ** (N - 1)) + ((N - 2) * X * Y * Z ** max(N - 3, 0) if N >= 3 else 0.0 * X)
    rho, c = coef[:, 0][:, None], coef[:, 1][:, None]
    r = ac.rhs(q)
    k = _interior(geo)
    assert k.sum() > 0
    np.testing.assert_allclose(r[k, 0], (-rho * c * c * div)[k], atol=1e-9)
    for i in range(3):
        np.testing.assert_allclose(r[k, 1 + i], (-dp[i] / rho)[k], atol=1e-9)


@pytest.mark.parametrize("N", [1, 3])
def test_elastic_polynomial_state_matches_pde(N):
    m, geo = _mesh(n=3, N=N)
    coef = di.elastic_loguniform(m, 8)
    el = ElasticOracle(geo, coef)
    X, Y, Z = (geo.xyz[..., i] for i in range(3))
    rng = np.random.default_rng(3)
    # each field: a random linear combination of x^N, y^N, z^N, x, y, z, 1
    A = rng.standard_normal((9, 7))
    basis = [X**N, Y**N, Z**N, X, Y, Z, np.ones_like(X)]
    dbasis = [  # d/dx, d/dy, d/dz of each basis function
        [N * X ** (N - 1), 0 * X, 0 * X],
        [0 * X, N * Y ** (N - 1), 0 * X],
        [0 * X, 0 * X, N * Z ** (N - 1)],
        [1 + 0 * X, 0 * X, 0 * X],
        [0 * X, 1 + 0 * X, 0 * X],
        [0 * X, 0 * X, 1 + 0 * X],
        [0 * X, 0 * X, 0 * X],
    ]
    q = np.stack([sum(A[f, b] * basis[b] for b in range(7)) for f in range(9)], 1)
    dq = [[sum(A[f, b] * dbasis[b][d] for b in range(7)) for d in range(3)] for f in range(9)]
    rho, lam, mu = (coef[:, i][:, None] for i in range(3))
    tix = {(i, j): a for a, (i, j) in enumerate(VOIGT)}
    tix.update({(j, i): a for a, (i, j) in enumerate(VOIGT)})
    divv = dq[0][0] + dq[1][1] + dq[2][2]
    r = el.rhs(q)
    k = _interior(geo)
    for i in range(3):
        divs = sum(dq[3 + tix[(i, j)]][j] for j in range(3))
        np.testing.assert_allclose(r[k, i], (divs / rho)[k], atol=1e-9)
    for a, (i, j) in enumerate(VOIGT):
        val = mu * (dq[i][j] + dq[j][i]) + (lam * divv if i == j else 0.0)
        np.testing.assert_allclose(r[k, 3 + a], val[k], atol=1e-9)


def _face_lift_of_constants(geo, per_face):
    """sum_f LIFT_f (per_face[k, f] * 1) -> (K, Np); per_face (K, 4)."""
    Nfp = geo.ref.Nfp
    flux = np.repeat(per_face[:, :, None], Nfp, axis=2)
    return flux.reshape(geo.K, 4 * Nfp) @ geo.ref.LIFT.T


@pytest.mark.parametrize("periodic", [False, True])
def test_acoustic_riemann_problem(periodic):
    m, geo = _mesh(n=3, periodic=periodic, N=3)
    coef = di.acoustic_loguniform(m, 11)
    ac = AcousticOracle(geo, coef)
    rng = np.random.default_rng(5)
    cell = rng.standard_normal((geo.K, 4))
    q = np.repeat(cell[:, :, None], geo.ref.Np, axis=2)
    rho, c = coef[:, 0], coef[:, 1]
    Z = rho * c
    n = geo.normals
    kn = np.where(geo.wall, np.arange(geo.K)[:, None], geo.EToE)
    pm, vm = cell[:, 0][:, None], np.einsum("kfi,ki->kf", n, cell[:, 1:4])
    pp, vp = cell[kn, 0], np.einsum("kfi,kfi->kf", n, cell[kn, 1:4])
    Zm, Zp = Z[:, None], Z[kn]
    pp = np.where(geo.wall, pm, pp)
    vp = np.where(geo.wall, -vm, vp)
    # characteristics: p + Z^- v_n carried out of the element, p - Z^+ v_n in
    vs = (pm - pp + Zm * vm + Zp * vp) / (Zm + Zp)
    ps = pm - Zm * (vs - vm)
    r = ac.rhs(q)
    Fs = geo.Fscale
    exp_p = _face_lift_of_constants(geo, Fs * (rho * c * c)[:, None] * (vm - vs))
    np.testing.assert_allclose(r[:, 0], exp_p, atol=1e-10)
    for i in range(3):
        exp_v = _face_lift_of_constants(geo, Fs * (pm - ps) * n[:, :, i] / rho[:, None])
        np.testing.assert_allclose(r[:, 1 + i], exp_v, atol=1e-10)


@pytest.mark.parametrize("periodic", [False, True])
def test_elastic_riemann_problem(periodic):
    m, geo = _mesh(n=3, periodic=periodic, N=2)
    coef = di.elastic_loguniform(m, 12)
    el = ElasticOracle(geo, coef)
    rng = np.random.default_rng(6)
    cell = rng.standard_normal((geo.K, 9))
    q = np.repeat(cell[:, :, None], geo.ref.Np, axis=2)
    rho, lam, mu = coef[:, 0], coef[:, 1], coef[:, 2]
    Zp = rho * np.sqrt((lam + 2 * mu) / rho)
    Zs = rho * np.sqrt(mu / rho)
    n = geo.normals
    kn = np.where(geo.wall, np.arange(geo.K)[:, None], geo.EToE)

    def full(s):  # (..., 6) -> (..., 3, 3)
        S = np.empty(s.shape[:-1] + (3, 3))
        for a, (i, j) in enumerate(VOIGT):
            S[..., i, j] = S[..., j, i] = s[..., a]
        return S

    vm = np.repeat(cell[:, None, 0:3], 4, 1)
    vp = cell[kn, 0:3]
    tm = np.einsum("kfij,kfj->kfi", full(np.repeat(cell[:, None, 3:9], 4, 1)), n)
    tp = np.einsum("kfij,kfj->kfi", full(cell[kn, 3:9]), n)
    w = geo.wall[..., None]
    vp = np.where(w, vm, vp)
    tp = np.where(w, -tm, tp)
    # normal part with P impedances, tangential part with S impedances
    Zpm, Zpp = Zp[:, None, None], np.where(geo.wall, Zp[:, None], Zp[kn])[..., None]
    Zsm, Zsp = Zs[:, None, None], np.where(geo.wall, Zs[:, None], Zs[kn])[..., None]
    nn = n

    def split(x):
        xn = np.einsum("kfi,kfi->kf", x, nn)[..., None]
        return xn, x - xn * nn

    vmn, vmt = split(vm)
    vpn, vpt = split(vp)
    tmn, tmt = split(tm)
    tpn, tpt = split(tp)
    # -s_nn plays the role of a pressure: v* = (Z^-v^- + Z^+v^+ + t^+ - t^-)/(Z^-+Z^+)
    vsn = (Zpm * vmn + Zpp * vpn + tpn - tmn) / (Zpm + Zpp)
    vst = (Zsm * vmt + Zsp * vpt + tpt - tmt) / (Zsm + Zsp)
    tsn = tmn + Zpm * (vsn - vmn)
    tst = tmt + Zsm * (vst - vmt)
    dv = (vsn - vmn) * nn + (vst - vmt)
    dt = (tsn - tmn) * nn + (tst - tmt)
    r = el.rhs(q)
    Fs = geo.Fscale
    for i in range(3):
        exp = _face_lift_of_constants(geo, Fs * dt[..., i] / rho[:, None])
        np.testing.assert_allclose(r[:, i], exp, atol=1e-10)
    dvn = np.einsum("kfi,kfi->kf", dv, nn)
    for a, (i, j) in enumerate(VOIGT):
        corr = mu[:, None] * (nn[..., i] * dv[..., j] + dv[..., i] * nn[..., j])
        if i == j:
            corr = corr + lam[:, None] * dvn
        exp = _face_lift_of_constants(geo, Fs * corr)
        np.testing.assert_allclose(r[:, 3 + a], exp, atol=1e-10)


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("N", [1, 3])
def test_energy_rate_nonpositive(physics, periodic, N):
    m, geo = _mesh(n=3, periodic=periodic, N=N)
    rng = np.random.default_rng(N + 10 * periodic)
    if physics == "acoustic":
        o = AcousticOracle(geo, di.acoustic_loguniform(m, 21))
    else:
        o = ElasticOracle(geo, di.elastic_loguniform(m, 22))
    for _ in range(3):
        q = rng.standard_normal((geo.K, o.nfields, geo.ref.Np))
        rate = o.energy_rate(q)
        assert rate < 0.0
        # a continuous state dissipates nothing on interior faces
    if periodic:
        X = geo.xyz[..., 0]
        q = np.zeros((geo.K, o.nfields, geo.ref.Np))
        q[:, 0] = 1.0
        assert abs(o.energy_rate(q)) < 1e-11


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("periodic", [False, True])
def test_rhs_invariant_under_vertex_relabelling(physics, periodic):
    """Listing each element's vertices in another even order changes no
    physical quantity: on a discontinuous state (a per-element phase, so every
    face carries a jump) the right-hand side at each physical node is the same,
    which pins the face-node pairing under all six orientations."""
    N = 3
    m = di.kuhn_box(3, periodic=periodic, jitter=0.1, seed=4)
    r = di.relabel_vertices(m, seed=3)
    g0 = build_mesh(N, m.elem_xyz, m.elem_topo, m.period)
    g1 = build_mesh(N, r.elem_xyz, r.elem_topo, r.period)
    # node i of element k in the original numbering is node pi[k, i] after relabelling
    dist = np.linalg.norm(g0.xyz[:, :, None, :] - g1.xyz[:, None, :, :], axis=-1)
    pi = dist.argmin(axis=2)
    assert dist.min(axis=2).max() < 1e-12
    nf = 4 if physics == "acoustic" else 9
    phase = np.random.Generator(np.random.PCG64(8)).uniform(0.0, 6.0, size=(m.K, nf))

    def state(x):
        return np.stack(
            [np.sin(phase[:, c, None] + 2.3 * x[..., 0] - 1.1 * x[..., 1] + (0.7 + 0.2 * c) * x[..., 2])
             for c in range(nf)], axis=1)

    coef = di.acoustic_loguniform(m, 1) if physics == "acoustic" else di.elastic_loguniform(m, 2)
    O = AcousticOracle if physics == "acoustic" else ElasticOracle
    r0 = O(g0, coef).rhs(state(g0.xyz))
    r1 = O(g1, coef).rhs(state(g1.xyz))
    r1_in_0 = r1[np.arange(m.K)[:, None, None], np.arange(nf)[None, :, None], pi[:, None, :]]
    np.testing.assert_allclose(r1_in_0, r0, atol=1e-10 * np.abs(r0).max())
