"""Seeded synthetic inputs for the tetrahedral DG wave solver.

This module is shared by the FP64 oracle and the GPU product path.  It holds
none of the discontinuous Galerkin arithmetic: only the synthetic workload
(Kuhn-split box meshes with optional vertex jitter, per-element material
coefficients, analytic initial-data functions of the physical coordinates and
a time-step recipe from raw vertex geometry), so that both sides are fed the
same inputs.

Mesh format (the product's set-up call takes the same arrays):

* ``elem_xyz``  float64 [K, 4, 3]  vertex coordinates of every tetrahedron
  (positively oriented: det[x2-x1, x3-x1, x4-x1] > 0);
* ``elem_topo`` int64   [K, 4]     topological vertex ids; two elements share
  a face iff they share the three ids of that face (periodic boxes identify
  opposite vertices through these ids, while ``elem_xyz`` keeps the unwrapped
  coordinates);
* ``period``    float64 [3] or None, the box lengths of a periodic mesh
  (0 along an axis that is not periodic).

Faces that have no partner are boundary faces (reflecting walls).
"""

from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

# ----------------------------------------------------------------------------
# Meshes
# ----------------------------------------------------------------------------


@dataclass
class TetMesh:
    elem_xyz: np.ndarray
    elem_topo: np.ndarray
    period: np.ndarray | None
    dims: tuple
    lengths: tuple

    @property
    def K(self) -> int:
        return int(self.elem_xyz.shape[0])


_PERMS = list(itertools.permutations(range(3)))


def kuhn_box(
    nx: int,
    ny: int | None = None,
    nz: int | None = None,
    lengths=(1.0, 1.0, 1.0),
    jitter: float = 0.0,
    seed: int = 0,
    periodic=False,
) -> TetMesh:
    """Box of nx*ny*nz subcubes, each split into 6 Kuhn tetrahedra.

    Each subcube is cut along its (0,0,0)-(1,1,1) diagonal into the six
    tetrahedra v0 -> v0+e_a -> v0+e_a+e_b -> v0+e_a+e_b+e_c, one per
    permutation (a, b, c) of the axes; the split is conforming across subcubes
    and compatible with periodic identification.  Elements are ordered
    subcube by subcube (x fastest), six consecutive elements per subcube.

    ``periodic`` is one flag for all axes or a triple of per-axis flags.
    ``jitter`` moves vertices by U[-jitter*h, jitter*h] per coordinate (h the
    subcube edge along that axis), consistently through the topological id;
    vertices on the boundary planes of a non-periodic axis stay fixed.  The
    draw is repeated with the next seed offset until every element is
    positively oriented.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    per_axis = tuple(bool(x) for x in (periodic if isinstance(periodic, (tuple, list)) else (periodic,) * 3))
    L = np.asarray(lengths, dtype=float)
    h = L / np.array([nx, ny, nz], dtype=float)
    gi, gj, gk = np.meshgrid(
        np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij"
    )
    grid = np.stack([gi, gj, gk], axis=-1).reshape(-1, 3)  # index order x slowest here

    K = 6 * nx * ny * nz
    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cell = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=-1)  # x fastest
    corners = np.zeros((cell.shape[0], 6, 4, 3), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        path = [cell.copy()]
        c = cell.copy()
        for ax in perm:
            c = c.copy()
            c[:, ax] += 1
            path.append(c)
        if np.linalg.det(np.eye(3)[list(perm)]) < 0:  # odd permutation
            path[2], path[3] = path[3], path[2]
        corners[:, p] = np.stack(path, axis=1)
    corners = corners.reshape(K, 4, 3)
    topo = _vectorised_ids(corners, nx, ny, nz, per_axis)

    base = corners.astype(float) * h  # unwrapped coordinates
    attempt = 0
    while True:
        xyz = base.copy()
        if jitter > 0.0:
            rng = np.random.Generator(np.random.PCG64(seed + 7919 * attempt))
            if all(per_axis):
                nv = nx * ny * nz
                d = rng.uniform(-jitter, jitter, size=(nv, 3)) * h
                xyz += d[topo]
            elif not any(per_axis):
                nv = (nx + 1) * (ny + 1) * (nz + 1)
                d = rng.uniform(-jitter, jitter, size=(nv, 3)) * h
                interior = (
                    (grid[:, 0] > 0) & (grid[:, 0] < nx)
                    & (grid[:, 1] > 0) & (grid[:, 1] < ny)
                    & (grid[:, 2] > 0) & (grid[:, 2] < nz)
                )
                d[~interior] = 0.0
                gid = (corners[..., 0] * (ny + 1) + corners[..., 1]) * (nz + 1) + corners[..., 2]
                xyz += d[gid]
            else:
                nv = int(topo.max()) + 1
                d = rng.uniform(-jitter, jitter, size=(nv, 3)) * h
                fixed = np.zeros(corners.shape[:-1], dtype=bool)
                for a, n_a in enumerate((nx, ny, nz)):
                    if not per_axis[a]:
                        fixed |= (corners[..., a] == 0) | (corners[..., a] == n_a)
                dv = d[topo]
                dv[fixed] = 0.0
                xyz += dv
        dets = np.linalg.det(
            np.stack([xyz[:, 1] - xyz[:, 0], xyz[:, 2] - xyz[:, 0], xyz[:, 3] - xyz[:, 0]], axis=-1)
        )
        if np.all(dets > 0.0):
            break
        attempt += 1
        if attempt > 50:
            raise RuntimeError("could not draw a valid jittered mesh")
    period = np.where(per_axis, L, 0.0) if any(per_axis) else None
    return TetMesh(
        elem_xyz=np.ascontiguousarray(xyz),
        elem_topo=np.ascontiguousarray(topo),
        period=period,
        dims=(nx, ny, nz),
        lengths=tuple(float(x) for x in L),
    )


def _vectorised_ids(corners, nx, ny, nz, per_axis):
    ids = []
    sizes = []
    for a, n_a in enumerate((nx, ny, nz)):
        c = corners[..., a]
        ids.append(c % n_a if per_axis[a] else c)
        sizes.append(n_a if per_axis[a] else n_a + 1)
    return (ids[0] * sizes[1] + ids[1]) * sizes[2] + ids[2]


_EVEN_PERMS4 = [
    p for p in itertools.permutations(range(4))
    if sum(1 for i in range(4) for j in range(i + 1, 4) if p[i] > p[j]) % 2 == 0
]


def relabel_vertices(mesh: TetMesh, seed: int) -> TetMesh:
    """The same mesh with every element's vertices listed in a random even order.

    An even permutation keeps each element positively oriented, and the
    physical mesh (and so the discrete solution, up to node numbering) is
    unchanged; only the local vertex numbering moves, which makes the shared
    faces of neighbours meet under all six relative orientations instead of
    the two that a Kuhn split produces.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = np.asarray(_EVEN_PERMS4, dtype=np.int64)[rng.integers(0, len(_EVEN_PERMS4), size=mesh.K)]
    rows = np.arange(mesh.K)[:, None]
    return TetMesh(
        elem_xyz=np.ascontiguousarray(mesh.elem_xyz[rows, pick]),
        elem_topo=np.ascontiguousarray(mesh.elem_topo[rows, pick]),
        period=mesh.period,
        dims=mesh.dims,
        lengths=mesh.lengths,
    )


def graded_kuhn_box(n_fine: int, n_coarse: int, split: float = 0.5, periodic=False) -> TetMesh:
    """Kuhn box on the unit cube graded along every axis: cells are
    split / n_fine wide below `split` and (1 - split) / n_coarse wide above,
    so the corner region [0, split)^3 holds the smallest elements and
    [split, 1]^3 the largest (a mesh for local time stepping); ``periodic``
    as in ``kuhn_box``."""
    n = n_fine + n_coarse
    base = kuhn_box(n, n, n, lengths=(float(n),) * 3, periodic=periodic)
    i = base.elem_xyz  # integer node indices (unwrapped)
    x = np.where(i <= n_fine, i * (split / n_fine), split + (i - n_fine) * ((1.0 - split) / n_coarse))
    period = None if base.period is None else np.where(base.period > 0, 1.0, 0.0)
    return TetMesh(elem_xyz=np.ascontiguousarray(x), elem_topo=base.elem_topo, period=period,
                   dims=base.dims, lengths=(1.0, 1.0, 1.0))


def permute_elements(mesh: TetMesh, order: np.ndarray) -> TetMesh:
    """The same mesh with element i of the result being element order[i]."""
    order = np.asarray(order, dtype=np.int64)
    return TetMesh(elem_xyz=np.ascontiguousarray(mesh.elem_xyz[order]),
                   elem_topo=np.ascontiguousarray(mesh.elem_topo[order]),
                   period=mesh.period, dims=mesh.dims, lengths=mesh.lengths)


def element_centroids(mesh: TetMesh) -> np.ndarray:
    return mesh.elem_xyz.mean(axis=1)


def inradius(mesh: TetMesh) -> np.ndarray:
    """Inradius 3V / (sum of face areas) of every element, from its vertices."""
    x = mesh.elem_xyz
    vol = np.abs(
        np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], -1))
    ) / 6.0
    area = np.zeros(len(x))
    for a, b, c in ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)):
        area += 0.5 * np.linalg.norm(np.cross(x[:, b] - x[:, a], x[:, c] - x[:, a]), axis=1)
    return 3.0 * vol / area


# ----------------------------------------------------------------------------
# Material coefficients
# ----------------------------------------------------------------------------


def acoustic_constant(mesh: TetMesh, rho: float = 1.0, c: float = 1.0) -> np.ndarray:
    """[K, 2] (rho, c) constant over the mesh."""
    out = np.empty((mesh.K, 2))
    out[:, 0] = rho
    out[:, 1] = c
    return out


def acoustic_two_layer(mesh: TetMesh, z_split: float = 0.5) -> np.ndarray:
    """[K, 2] (rho, c): (1, 1) below the plane z = z_split, (2, 1.5) above,
    chosen by element centroid."""
    zc = element_centroids(mesh)[:, 2]
    out = np.empty((mesh.K, 2))
    low = zc < z_split
    out[low] = (1.0, 1.0)
    out[~low] = (2.0, 1.5)
    return out


def acoustic_loguniform(mesh: TetMesh, seed: int, lo: float = 0.5, hi: float = 2.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=(mesh.K, 2)))


def elastic_constant(mesh: TetMesh, rho=1.0, lam=1.0, mu=1.0) -> np.ndarray:
    out = np.empty((mesh.K, 3))
    out[:] = (rho, lam, mu)
    return out


def elastic_loguniform(mesh: TetMesh, seed: int, lo: float = 0.5, hi: float = 2.0) -> np.ndarray:
    """[K, 3] (rho, lambda, mu), each exp(U[ln lo, ln hi]) independently."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=(mesh.K, 3)))


ANISO_UPPER6 = [(a, b) for a in range(6) for b in range(a, 6)]  # order of the 21 stiffness entries


def anisotropic_random(mesh: TetMesh, seed: int, strength: float = 0.35) -> np.ndarray:
    """Per element (rho, 21 upper-triangle entries of a symmetric positive
    definite Voigt stiffness C): an isotropic stiffness with lambda, mu
    log-uniform on [1/2, 2] plus a seeded symmetric perturbation of relative
    size `strength`, redrawn (for the elements that need it, in rounds) until
    C is positive definite with its smallest eigenvalue at least a tenth of
    mu; rho log-uniform on [1/2, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho, lam, mu = np.exp(rng.uniform(np.log(0.5), np.log(2.0), (mesh.K, 3))).T
    base = np.zeros((mesh.K, 6, 6))
    base[:, :3, :3] = lam[:, None, None]
    d = np.arange(3)
    base[:, d, d] = (lam + 2 * mu)[:, None]
    base[:, d + 3, d + 3] = mu[:, None]
    C = np.empty_like(base)
    todo = np.arange(mesh.K)
    while todo.size:
        R = rng.standard_normal((todo.size, 6, 6))
        Ct = base[todo] + (strength * (lam + 2 * mu)[todo] * 0.5 / 6.0)[:, None, None] * (R + np.swapaxes(R, 1, 2))
        ok = np.linalg.eigvalsh(Ct).min(axis=1) >= 0.1 * mu[todo]
        C[todo[ok]] = Ct[ok]
        todo = todo[~ok]
    out = np.zeros((mesh.K, 22))
    out[:, 0] = rho
    for i, (a, b) in enumerate(ANISO_UPPER6):
        out[:, 1 + i] = C[:, a, b]
    return out


def anisotropic_from_isotropic(coef_iso: np.ndarray) -> np.ndarray:
    """(rho, lambda, mu) rows -> (rho, 21 stiffness entries) of the same medium."""
    out = np.zeros((coef_iso.shape[0], 22))
    for k, (rho, lam, mu) in enumerate(np.asarray(coef_iso, dtype=float)):
        C = np.zeros((6, 6))
        C[:3, :3] = lam
        C[np.arange(3), np.arange(3)] = lam + 2 * mu
        C[np.arange(3, 6), np.arange(3, 6)] = mu
        out[k, 0] = rho
        out[k, 1:] = [C[a, b] for a, b in ANISO_UPPER6]
    return out


def _stiffness(c21):
    C = np.zeros((6, 6))
    for i, (a, b) in enumerate(ANISO_UPPER6):
        C[a, b] = C[b, a] = c21[i]
    return C


def anisotropic_speed_bound(coef: np.ndarray) -> np.ndarray:
    """Per element sqrt(lambda_max(C in Mandel form) / rho), an upper bound of
    every wave speed in every direction (for the time step)."""
    D = np.diag([1, 1, 1, math.sqrt(2), math.sqrt(2), math.sqrt(2)])
    return np.array([math.sqrt(np.linalg.eigvalsh(D @ _stiffness(row[1:]) @ D).max() / row[0])
                     for row in np.asarray(coef, dtype=float)])


def anisotropic_plane_wave(x, m, rho, c21, mode: int = 0, t: float = 0.0) -> np.ndarray:
    """Fields [9, ...] of a plane wave along the integer vector m in a
    homogeneous anisotropic medium: (c^2, d) the mode-th eigenpair (ascending)
    of the Christoffel matrix G_ik = C_ijkl m_j m_l / rho for the unit m,
    v = d f, s = -C : sym(m (x) d) f / c, f = cos(2 pi (m.x) - 2 pi |m| c t)."""
    m = np.asarray(m, dtype=float)
    km = np.linalg.norm(m)
    mh = m / km
    C = _stiffness(c21)
    eps_basis = lambda d: np.array([mh[0] * d[0], mh[1] * d[1], mh[2] * d[2], mh[1] * d[2] + mh[2] * d[1],
                                    mh[0] * d[2] + mh[2] * d[0], mh[0] * d[1] + mh[1] * d[0]])
    Gam = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        sv = C @ eps_basis(e)  # stress (Voigt) of sym(m (x) e_k)
        S = np.array([[sv[0], sv[5], sv[4]], [sv[5], sv[1], sv[3]], [sv[4], sv[3], sv[2]]])
        Gam[:, k] = S @ mh / rho
    w, V = np.linalg.eigh(0.5 * (Gam + Gam.T))
    c = math.sqrt(w[mode])
    d = V[:, mode]
    f = np.cos(2.0 * math.pi * (x @ m) - 2.0 * math.pi * km * c * t)
    out = np.zeros((9,) + f.shape)
    for i in range(3):
        out[i] = d[i] * f
    sv = -(C @ eps_basis(d)) / c
    for a in range(6):
        out[3 + a] = sv[a] * f
    return out


def max_wave_speed(coef: np.ndarray, physics: str) -> float:
    if physics == "acoustic":
        return float(np.max(coef[:, 1]))
    if physics == "anisotropic":
        return float(np.max(anisotropic_speed_bound(coef)))
    rho, lam, mu = coef[:, 0], coef[:, 1], coef[:, 2]
    return float(np.max(np.sqrt((lam + 2.0 * mu) / rho)))


# ----------------------------------------------------------------------------
# Initial data (analytic functions of the physical coordinates)
# ----------------------------------------------------------------------------

ACOUSTIC_FIELDS = ("p", "u", "v", "w")
ELASTIC_FIELDS = ("vx", "vy", "vz", "sxx", "syy", "szz", "syz", "sxz", "sxy")


def gaussian(x: np.ndarray, center=(0.5, 0.5, 0.5), sigma: float = 0.1) -> np.ndarray:
    d = x - np.asarray(center, dtype=float)
    return np.exp(-np.sum(d * d, axis=-1) / (2.0 * sigma * sigma))


def acoustic_gaussian(x: np.ndarray, center=(0.5, 0.5, 0.5), sigma=0.1) -> np.ndarray:
    """Fields [4, ...]: p = Gaussian pulse, v = 0.  x has shape [..., 3]."""
    out = np.zeros((4,) + x.shape[:-1])
    out[0] = gaussian(x, center, sigma)
    return out


def elastic_gaussian(x: np.ndarray, center=(0.5, 0.5, 0.5), sigma=0.1) -> np.ndarray:
    """Fields [9, ...]: v = Gaussian * (1,1,1)/sqrt(3), sigma = 0."""
    out = np.zeros((9,) + x.shape[:-1])
    g = gaussian(x, center, sigma) / math.sqrt(3.0)
    out[0] = out[1] = out[2] = g
    return out


def gaussian_pulses(x: np.ndarray, nfields: int, seed: int = 7, sigma: float = 0.1) -> np.ndarray:
    """Fields [nfields, ...]: field c is a Gaussian pulse of width sigma and
    amplitude 1 + 0.3 c centred at a seeded point of [0.3, 0.7]^3, so that
    every field carries the pulse's length scale (a state in which no field
    vanishes, for per-field error norms)."""
    centres = np.random.default_rng(seed).uniform(0.3, 0.7, (nfields, 3))
    return np.stack([(1.0 + 0.3 * c) * gaussian(x, centres[c], sigma) for c in range(nfields)])


def acoustic_plane_wave(x, m, rho=1.0, c=1.0, t=0.0) -> np.ndarray:
    """Travelling acoustic plane wave p = cos(2 pi m.x - omega t), omega =
    2 pi |m| c, v = mhat p / (rho c): an exact solution of the pressure-velocity
    system in a homogeneous medium (periodic for integer m on a unit box)."""
    m = np.asarray(m, dtype=float)
    km = np.linalg.norm(m)
    mh = m / km
    ph = 2.0 * math.pi * (x @ m) - 2.0 * math.pi * km * c * t
    f = np.cos(ph)
    out = np.zeros((4,) + x.shape[:-1])
    out[0] = f
    for i in range(3):
        out[1 + i] = mh[i] * f / (rho * c)
    return out


def _sym_to_voigt(S):
    """Symmetric 3x3 (leading dims) -> (xx, yy, zz, yz, xz, xy)."""
    return np.stack([S[0, 0], S[1, 1], S[2, 2], S[1, 2], S[0, 2], S[0, 1]])


def elastic_plane_wave(x, m, kind="P", rho=1.0, lam=1.0, mu=1.0, t=0.0, d=None) -> np.ndarray:
    """Elastic plane waves in a homogeneous isotropic medium.

    P: v = mhat f, sigma = -(lam I + 2 mu mhat mhat^T) f / c_p;
    S: v = d f (d unit, d . mhat = 0), sigma = -(mu/c_s)(mhat d^T + d mhat^T) f;
    f = cos(2 pi m.x - omega t) with omega = 2 pi |m| c_p (resp. c_s).
    """
    m = np.asarray(m, dtype=float)
    km = np.linalg.norm(m)
    mh = m / km
    cp = math.sqrt((lam + 2.0 * mu) / rho)
    cs = math.sqrt(mu / rho)
    out = np.zeros((9,) + x.shape[:-1])
    if kind == "P":
        f = np.cos(2.0 * math.pi * (x @ m) - 2.0 * math.pi * km * cp * t)
        for i in range(3):
            out[i] = mh[i] * f
        S = -(lam * np.eye(3) + 2.0 * mu * np.outer(mh, mh)) / cp
    else:
        if d is None:
            trial = np.array([1.0, 0.0, 0.0]) if abs(mh[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
            d = trial - (trial @ mh) * mh
        d = np.asarray(d, float)
        d = d / np.linalg.norm(d)
        f = np.cos(2.0 * math.pi * (x @ m) - 2.0 * math.pi * km * cs * t)
        for i in range(3):
            out[i] = d[i] * f
        S = -(mu / cs) * (np.outer(mh, d) + np.outer(d, mh))
    V = _sym_to_voigt(S)
    for a in range(6):
        out[3 + a] = V[a] * f
    return out


# ----------------------------------------------------------------------------
# Time step recipe and the paper-scale workloads
# ----------------------------------------------------------------------------

CFL_DEFAULT = 0.5


def time_step(mesh: TetMesh, N: int, cmax: float, cfl: float = CFL_DEFAULT) -> float:
    """dt = cfl * min inradius / (cmax * (N+1)^2), from raw vertex geometry."""
    return float(cfl * inradius(mesh).min() / (cmax * (N + 1) ** 2))


def local_time_steps(mesh: TetMesh, N: int, c_elem: np.ndarray, cfl: float = CFL_DEFAULT) -> np.ndarray:
    """Per-element step cfl * inradius_k / (c_k (N+1)^2), the recipe of
    ``time_step`` element by element (c_k: the element's fastest speed)."""
    return cfl * inradius(mesh) / (np.asarray(c_elem, dtype=float) * (N + 1) ** 2)


def two_rate_classes(mesh: TetMesh, N: int, c_elem: np.ndarray, cfl: float = CFL_DEFAULT):
    """(fast mask, macro step): the macro step is twice the smallest local
    step, and an element is fast when its local step is below the macro
    step (it then takes two half steps)."""
    dtk = local_time_steps(mesh, N, c_elem, cfl)
    dt = 2.0 * float(dtk.min())
    return dtk < dt, dt


def element_wave_speeds(coef: np.ndarray, physics: str) -> np.ndarray:
    """Fastest wave speed of every element (c, or c_p = sqrt((lam + 2 mu)/rho))."""
    coef = np.asarray(coef, dtype=float)
    if physics == "acoustic":
        return coef[:, 1]
    if physics == "anisotropic":
        return anisotropic_speed_bound(coef)
    return np.sqrt((coef[:, 1] + 2.0 * coef[:, 2]) / coef[:, 0])


def n_nodes(N: int) -> int:
    return (N + 1) * (N + 2) * (N + 3) // 6


def paper_scale_n(N: int, target_nodes: float = 2.0e6) -> int:
    """Subcubes per edge so that 6 n^3 N_p is closest to ~2M nodes."""
    return int(round((target_nodes / (6.0 * n_nodes(N))) ** (1.0 / 3.0)))


def batch_recipe(count: int = 64, seed: int = 2, k_lo: float = 2.0e3, k_hi: float = 2.0e5,
                 degrees=(2, 3, 4, 5, 6), n_lo: int = 7, n_hi: int = 32):
    """Independent meshes of uneven size and degree for batched stepping.

    Per mesh: K drawn log-uniform on [k_lo, k_hi] and snapped to the nearest
    Kuhn box 6 n^3 with n in [n_lo, n_hi]; degree uniform over `degrees`;
    its own jitter and coefficient seeds.  Returns a list of dicts with keys
    n, K, N, mesh_seed, coef_seed.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        k = float(np.exp(rng.uniform(np.log(k_lo), np.log(k_hi))))
        n = int(np.clip(round((k / 6.0) ** (1.0 / 3.0)), n_lo, n_hi))
        N = int(rng.choice(np.asarray(degrees)))
        out.append({"n": n, "K": 6 * n ** 3, "N": N, "mesh_seed": 1000 + i, "coef_seed": 2000 + i})
    return out
