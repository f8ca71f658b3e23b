"""Reference tetrahedron for the FP64 oracle (test infrastructure only).

Follows Sec. 2.2 of the paper: nodal Lagrange expansion (eq. (1)) at
warp-and-blend nodes with N_p = (N+1)(N+2)(N+3)/6 nodes, reference
differentiation matrices D_j and the merged lift matrix L (eqs. (3), (5)-(6)).
The paper defers the definitions of D_j and L to earlier work; the reading used
here is the standard nodal construction:

* orthonormal (Proriol-Koornwinder-Dubiner) basis psi_m on the tetrahedron,
  Vandermonde V[n, m] = psi_m(node_n);
* D_j = V_j V^{-1} with V_j[n, m] = d psi_m / d r_j (node_n);
* mass matrix M = (V V^T)^{-1};
* face mass E_f = (V2 V2^T)^{-1} with the orthonormal triangle basis on the
  face nodes, the face parameterised by the 2D reference triangle
  T = {(-1,-1), (1,-1), (-1,1)} (area 2);
* merged lift L = M^{-1} [E_1 .. E_4] (N_p x 4 N_fp), each E_f embedded at
  the volume rows of face f.

Conventions (shared with the product only through the documented interface):

* reference vertices v1=(-1,-1,-1), v2=(1,-1,-1), v3=(-1,1,-1), v4=(-1,-1,1);
  barycentrics l1 = -(1+r+s+t)/2, l2 = (1+r)/2, l3 = (1+s)/2, l4 = (1+t)/2;
* node n <-> integer lattice (l1,l2,l3,l4)*N, ordered with l4 outermost,
  then l3, then l2 innermost;
* faces (local vertex triples): f0 = (v1,v2,v3) [t=-1], f1 = (v1,v2,v4)
  [s=-1], f2 = (v2,v3,v4) [r+s+t=-1], f3 = (v1,v3,v4) [r=-1];
* face node j <-> (a, b) = N*(l of 2nd face vertex, l of 3rd face vertex),
  ordered with b outermost, a innermost.

Node placement (warp & blend, alpha = 0): see ``warp_blend_nodes``.
"""

from __future__ import annotations

import functools
import math
from dataclasses import dataclass

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import eval_jacobi, gammaln

FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))
# Unnormalised outward reference normals (gradient of the face's level-set
# function), consistent with the triangle T parameterisation of area 2.
REF_FACE_NORMALS = np.array(
    [[0.0, 0.0, -1.0], [0.0, -1.0, 0.0], [1.0, 1.0, 1.0], [-1.0, 0.0, 0.0]]
)
REF_VERTS = np.array(
    [[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]]
)


def n_nodes(N: int) -> int:
    return (N + 1) * (N + 2) * (N + 3) // 6


def n_face_nodes(N: int) -> int:
    return (N + 1) * (N + 2) // 2


def volume_lattice(N: int) -> np.ndarray:
    """Integer barycentric lattice (l1, l2, l3, l4), sum N, in node order."""
    pts = []
    for k in range(N + 1):
        for j in range(N + 1 - k):
            for i in range(N + 1 - j - k):
                pts.append((N - i - j - k, i, j, k))
    return np.array(pts, dtype=np.int64)


def face_lattice(N: int) -> np.ndarray:
    """Face lattice (a, b) in canonical face-node order (b outer, a inner)."""
    pts = []
    for b in range(N + 1):
        for a in range(N + 1 - b):
            pts.append((a, b))
    return np.array(pts, dtype=np.int64)


def face_masks(N: int) -> np.ndarray:
    """Fmask[f, j] = volume node index of face node j of face f."""
    lat = volume_lattice(N)
    lookup = {tuple(p): n for n, p in enumerate(lat)}
    fl = face_lattice(N)
    fm = np.zeros((4, len(fl)), dtype=np.int64)
    for f, (v0, v1, v2) in enumerate(FACE_VERTS):
        for j, (a, b) in enumerate(fl):
            bary = [0, 0, 0, 0]
            bary[v0] = N - a - b
            bary[v1] = a
            bary[v2] = b
            fm[f, j] = lookup[tuple(bary)]
    return fm


# ----------------------------------------------------------------------------
# 1D Gauss-Lobatto-Legendre points and the warp function
# ----------------------------------------------------------------------------

def gll_points(N: int) -> np.ndarray:
    """N+1 Gauss-Lobatto-Legendre points on [-1, 1]: +-1 and roots of P_N'."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = npleg.Legendre.basis(N).deriv().roots()
    x = np.concatenate([[-1.0], np.sort(inner.real), [1.0]])
    return x


def warp_factor(N: int, r: np.ndarray) -> np.ndarray:
    """Warp factor w(r)/(1-r^2), w = interpolated GLL-minus-equidistant shift.

    w(r) = sum_i (x_i^GLL - x_i^eq) l_i^eq(r), with l_i^eq the Lagrange
    polynomials on the N+1 equidistant points; the factor is zero at |r| = 1.
    """
    r = np.asarray(r, dtype=float)
    xg = gll_points(N)
    xe = np.linspace(-1.0, 1.0, N + 1)
    w = np.zeros_like(r)
    for i in range(N + 1):
        li = np.ones_like(r)
        for m in range(N + 1):
            if m != i:
                li = li * (r - xe[m]) / (xe[i] - xe[m])
        w = w + (xg[i] - xe[i]) * li
    out = np.zeros_like(r)
    inside = np.abs(r) < 1.0 - 1e-12
    out[inside] = w[inside] / (1.0 - r[inside] ** 2)
    return out


def warp_1d(N: int, r: np.ndarray) -> np.ndarray:
    """The edge displacement itself, w(r) (no division)."""
    r = np.asarray(r, dtype=float)
    return warp_factor(N, r) * (1.0 - r**2)


# ----------------------------------------------------------------------------
# Warp & blend nodes on the tetrahedron
# ----------------------------------------------------------------------------

_EQUI = np.array(
    [
        [-1.0, -1.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
        [1.0, -1.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
        [0.0, 2.0 / math.sqrt(3.0), -1.0 / math.sqrt(6.0)],
        [0.0, 0.0, 3.0 / math.sqrt(6.0)],
    ]
)


def warp_blend_nodes(N: int) -> np.ndarray:
    """Warp-and-blend nodes (r, s, t) in node order, alpha = 0.

    Construction on the equilateral tetrahedron with edge length 2:

    * equidistant lattice point X0 = sum_i L_i E_i (L = lattice / N);
    * a node on an edge PQ (two barycentrics zero) moves by the 1D warp
      w(L_Q - L_P) along the unit edge direction;
    * any other node moves by sum over faces F=(A,B,C) with opposite vertex D
      of  b_F * d_F, where the face displacement is
      d_F = sum over edges PQ of F of 4 L_P L_Q w(L_Q-L_P)/(1-(L_Q-L_P)^2)
      times the unit direction (E_Q-E_P)/2, and the blend is
      b_F = L_A L_B L_C / ((L_A + L_D/2)(L_B + L_D/2)(L_C + L_D/2)).
    The displaced point is mapped back to the reference tetrahedron through
    its barycentric coordinates.
    """
    lat = volume_lattice(N)
    if N == 0:
        return np.array([[-0.5, -0.5, -0.5]])
    L = lat.astype(float) / N
    X = L @ _EQUI
    shift = np.zeros_like(X)
    zero = lat == 0
    nzero = zero.sum(axis=1)
    for n in range(len(lat)):
        if nzero[n] == 3:  # vertex
            continue
        if nzero[n] == 2:  # edge node
            P, Q = [i for i in range(4) if not zero[n, i]]
            rr = L[n, Q] - L[n, P]
            shift[n] = warp_1d(N, np.array([rr]))[0] * (_EQUI[Q] - _EQUI[P]) / 2.0
            continue
        for F, (A, B, C) in enumerate(FACE_VERTS):
            D = ({0, 1, 2, 3} - {A, B, C}).pop()
            num = L[n, A] * L[n, B] * L[n, C]
            if num == 0.0:
                continue
            den = (
                (L[n, A] + 0.5 * L[n, D])
                * (L[n, B] + 0.5 * L[n, D])
                * (L[n, C] + 0.5 * L[n, D])
            )
            blend = num / den
            dF = np.zeros(3)
            for P, Q in ((A, B), (B, C), (A, C)):
                rr = L[n, Q] - L[n, P]
                dF += (
                    4.0
                    * L[n, P]
                    * L[n, Q]
                    * warp_factor(N, np.array([rr]))[0]
                    * (_EQUI[Q] - _EQUI[P])
                    / 2.0
                )
            shift[n] += blend * dF
    X = X + shift
    # barycentrics w.r.t. the equilateral tetrahedron
    Amat = np.vstack([_EQUI.T, np.ones(4)])
    bary = np.linalg.solve(Amat, np.vstack([X.T, np.ones(len(X))])).T
    return bary @ REF_VERTS


# ----------------------------------------------------------------------------
# Orthonormal bases
# ----------------------------------------------------------------------------

def jacobi_normalised(n: int, alpha: float, beta: float, x: np.ndarray) -> np.ndarray:
    """Jacobi P_n^(alpha,beta) scaled to unit norm in the weight (1-x)^a(1+x)^b."""
    lg = (
        (alpha + beta + 1.0) * math.log(2.0)
        - math.log(2 * n + alpha + beta + 1.0)
        + gammaln(n + alpha + 1.0)
        + gammaln(n + beta + 1.0)
        - gammaln(n + alpha + beta + 1.0)
        - gammaln(n + 1.0)
    )
    return eval_jacobi(n, alpha, beta, x) / math.exp(0.5 * lg)


def jacobi_normalised_deriv(n: int, alpha: float, beta: float, x: np.ndarray) -> np.ndarray:
    """d/dx of the normalised Jacobi polynomial.

    Uses d/dx P_n^(a,b) = (n+a+b+1)/2 P_{n-1}^(a+1,b+1) and rescales to the
    normalised family.
    """
    x = np.asarray(x, dtype=float)
    if n == 0:
        return np.zeros_like(x)
    lg_n = (
        (alpha + beta + 1.0) * math.log(2.0)
        - math.log(2 * n + alpha + beta + 1.0)
        + gammaln(n + alpha + 1.0)
        + gammaln(n + beta + 1.0)
        - gammaln(n + alpha + beta + 1.0)
        - gammaln(n + 1.0)
    )
    raw = 0.5 * (n + alpha + beta + 1.0) * eval_jacobi(n - 1, alpha + 1.0, beta + 1.0, x)
    return raw / math.exp(0.5 * lg_n)


def tet_basis_indices(N: int):
    return [(i, j, k) for i in range(N + 1) for j in range(N + 1 - i) for k in range(N + 1 - i - j)]


def collapsed_coords(r, s, t):
    """(a, b, c) collapsed coordinates; the singular limits take a=-1, b=-1."""
    r, s, t = (np.asarray(v, dtype=float) for v in (r, s, t))
    a = np.full_like(r, -1.0)
    den = -(s + t)
    ok = np.abs(den) > 1e-14
    a[ok] = 2.0 * (1.0 + r[ok]) / den[ok] - 1.0
    b = np.full_like(r, -1.0)
    ok = np.abs(1.0 - t) > 1e-14
    b[ok] = 2.0 * (1.0 + s[ok]) / (1.0 - t[ok]) - 1.0
    return a, b, t.copy()


def tet_basis(N: int, r, s, t) -> np.ndarray:
    """V[n, m] = psi_m(r_n, s_n, t_n), orthonormal on the reference tet.

    psi_ijk = 2 sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i P_k^(2i+2j+2,0)(c) (1-c)^(i+j).
    """
    a, b, c = collapsed_coords(r, s, t)
    cols = []
    for i, j, k in tet_basis_indices(N):
        cols.append(
            2.0
            * math.sqrt(2.0)
            * jacobi_normalised(i, 0.0, 0.0, a)
            * jacobi_normalised(j, 2 * i + 1.0, 0.0, b)
            * (1.0 - b) ** i
            * jacobi_normalised(k, 2 * i + 2 * j + 2.0, 0.0, c)
            * (1.0 - c) ** (i + j)
        )
    return np.stack(cols, axis=1)


def tet_basis_grad(N: int, r, s, t):
    """(Vr, Vs, Vt): derivatives of the orthonormal basis at the points.

    Chain rule through the collapsed coordinates, with the negative powers of
    (1-b) and (1-c) cancelled analytically (they only appear multiplied by a
    factor that vanishes when the exponent would be negative):

      d/dr = 8 sqrt2 fa' g (1-b)^(i-1) h (1-c)^(i+j-1)
      d/ds = 4 sqrt2 (1+a) fa' g (1-b)^(i-1) h (1-c)^(i+j-1)
           + 4 sqrt2 fa [g'(1-b)^i - i g (1-b)^(i-1)] h (1-c)^(i+j-1)
      d/dt = 4 sqrt2 (1+a) fa' g (1-b)^(i-1) h (1-c)^(i+j-1)
           + 2 sqrt2 (1+b) fa [g'(1-b)^i - i g (1-b)^(i-1)] h (1-c)^(i+j-1)
           + 2 sqrt2 fa g (1-b)^i [h'(1-c)^(i+j) - (i+j) h (1-c)^(i+j-1)]
    """
    a, b, c = collapsed_coords(r, s, t)
    s2 = math.sqrt(2.0)

    def pw(x, e):
        return x**e if e >= 0 else np.zeros_like(x)

    Vr, Vs, Vt = [], [], []
    for i, j, k in tet_basis_indices(N):
        fa = jacobi_normalised(i, 0.0, 0.0, a)
        dfa = jacobi_normalised_deriv(i, 0.0, 0.0, a)
        gb = jacobi_normalised(j, 2 * i + 1.0, 0.0, b)
        dgb = jacobi_normalised_deriv(j, 2 * i + 1.0, 0.0, b)
        hc = jacobi_normalised(k, 2 * i + 2 * j + 2.0, 0.0, c)
        dhc = jacobi_normalised_deriv(k, 2 * i + 2 * j + 2.0, 0.0, c)
        ob, oc = 1.0 - b, 1.0 - c
        # terms carrying fa' (vanish for i = 0)
        if i >= 1:
            ta = dfa * gb * pw(ob, i - 1) * hc * pw(oc, i + j - 1)
        else:
            ta = np.zeros_like(a)
        # terms carrying d/db of g (1-b)^i (vanish for i + j = 0)
        if i + j >= 1:
            gpart = dgb * pw(ob, i) - (i * gb * pw(ob, i - 1) if i >= 1 else 0.0)
            tb = fa * gpart * hc * pw(oc, i + j - 1)
        else:
            tb = np.zeros_like(a)
        hpart = dhc * pw(oc, i + j) - ((i + j) * hc * pw(oc, i + j - 1) if i + j >= 1 else 0.0)
        tc = fa * gb * pw(ob, i) * hpart
        Vr.append(8.0 * s2 * ta)
        Vs.append(4.0 * s2 * (1.0 + a) * ta + 4.0 * s2 * tb)
        Vt.append(4.0 * s2 * (1.0 + a) * ta + 2.0 * s2 * (1.0 + b) * tb + 2.0 * s2 * tc)
    return np.stack(Vr, 1), np.stack(Vs, 1), np.stack(Vt, 1)


def tri_basis(N: int, x, y) -> np.ndarray:
    """Orthonormal basis on T: sqrt2 P_i(a) P_j^(2i+1,0)(b) (1-b)^i."""
    x, y = np.asarray(x, float), np.asarray(y, float)
    a = np.full_like(x, -1.0)
    ok = np.abs(1.0 - y) > 1e-14
    a[ok] = 2.0 * (1.0 + x[ok]) / (1.0 - y[ok]) - 1.0
    b = y
    cols = []
    for i in range(N + 1):
        for j in range(N + 1 - i):
            cols.append(
                math.sqrt(2.0)
                * jacobi_normalised(i, 0.0, 0.0, a)
                * jacobi_normalised(j, 2 * i + 1.0, 0.0, b)
                * (1.0 - b) ** i
            )
    return np.stack(cols, axis=1)


# ----------------------------------------------------------------------------
# The reference element
# ----------------------------------------------------------------------------

@dataclass
class RefElement:
    N: int
    Np: int
    Nfp: int
    r: np.ndarray  # (Np, 3) node coordinates (r, s, t)
    lattice: np.ndarray  # (Np, 4)
    V: np.ndarray  # (Np, Np)
    D: np.ndarray  # (3, Np, Np): D[j] = d/dr_j
    M: np.ndarray  # (Np, Np) mass matrix on the reference tet
    Minv: np.ndarray
    Fmask: np.ndarray  # (4, Nfp)
    Eface: np.ndarray  # (Nfp, Nfp) face mass in T coordinates (same for all faces)
    LIFT: np.ndarray  # (Np, 4*Nfp)
    face_xy: np.ndarray  # (Nfp, 2) face nodes in T coordinates


@functools.lru_cache(maxsize=None)
def reference_element(N: int) -> RefElement:
    if not 1 <= N <= 10:
        raise ValueError("degree out of range")
    Np, Nfp = n_nodes(N), n_face_nodes(N)
    rst = warp_blend_nodes(N)
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    V = tet_basis(N, r, s, t)
    Vr, Vs, Vt = tet_basis_grad(N, r, s, t)
    Vinv = np.linalg.inv(V)
    D = np.stack([Vr @ Vinv, Vs @ Vinv, Vt @ Vinv])
    Minv = V @ V.T
    M = np.linalg.inv(Minv)
    Fmask = face_masks(N)
    lat = volume_lattice(N)
    # Face 0 lies in t = -1 with vertices v1, v2, v3, so its (r, s) are its T
    # coordinates.  The node set is symmetric under the tetrahedron's
    # symmetry group, so every face's nodes sit at the same T coordinates
    # through that face's own vertex order (checked by the tests), and one
    # face mass matrix serves all four faces.
    face_xy = rst[Fmask[0]][:, :2]
    V2 = tri_basis(N, face_xy[:, 0], face_xy[:, 1])
    Eface = np.linalg.inv(V2 @ V2.T)
    E = np.zeros((Np, 4 * Nfp))
    for f in range(4):
        E[np.ix_(Fmask[f], np.arange(f * Nfp, (f + 1) * Nfp))] = Eface
    LIFT = Minv @ E
    return RefElement(
        N=N, Np=Np, Nfp=Nfp, r=rst, lattice=lat, V=V, D=D, M=M, Minv=Minv,
        Fmask=Fmask, Eface=Eface, LIFT=LIFT, face_xy=face_xy,
    )


def face_param_coords(N: int, f: int) -> np.ndarray:
    """T coordinates of face f's nodes through its own vertex order.

    Face node j of face f with face barycentrics (l_A, l_B, l_C) (A, B, C the
    face's vertices in order) sits at l_A (-1,-1) + l_B (1,-1) + l_C (-1,1).
    """
    ref = reference_element(N)
    A, B, C = FACE_VERTS[f]
    rst = ref.r[ref.Fmask[f]]
    lam = np.stack(
        [-(1 + rst.sum(1)) / 2, (1 + rst[:, 0]) / 2, (1 + rst[:, 1]) / 2, (1 + rst[:, 2]) / 2], 1
    )
    Tv = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
    return lam[:, [A, B, C]] @ Tv
