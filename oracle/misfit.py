"""Point source, receivers, L2 misfit and its coefficient gradient (FP64 oracle).

Test infrastructure only.  The paper stops at the forward step; this module
defines the inverse-problem functional that the adjoint path differentiates,
as plain definitions on top of the forward oracle:

* point location: the element k whose barycentric coordinates of x are all
  >= -tol (the first such element), and the reference coordinates
  xi = F^{-1} (x - x1) - 1 of the affine map x(r) = x1 + F (r + 1);
* nodal interpolation at xi: u(xi) = l(xi) . u_nodes with the Lagrange
  weights l(xi) = V^{-T} psi(xi), psi the orthonormal basis (Sec. 2.2,
  eq. (1));
* point source: r^m gains f(t_m) b with b = (1/J_k) M^{-1} l(xi_s) in the
  source fields (acoustic: p; elastic: the three normal stresses, an
  explosive source), i.e. the Galerkin projection of f(t) delta(x - x_s);
  t_m = m dt and the source enters the Adams-Bashforth history like the
  rest of r;
* Ricker wavelet f(t) = (1 - 2 a) exp(-a), a = (pi f0 (t - t0))^2;
* receivers: u_r(t_m) = l(xi_r) . q_{k_r, c} for the recorded fields
  (acoustic: p; elastic: v1, v2, v3);
* misfit J = 1/2 dt sum_{m=1..M} sum_channels (u(t_m) - d(t_m))^2 from the
  zero initial state.

The reference gradient dJ/dtheta with respect to every per-element
coefficient is the complex-step derivative Im J(theta + i h e) / h: J is a
real-analytic function of the coefficients (rational functions and square
roots of positive numbers), so the complex step is exact to rounding and has
no subtractive cancellation.  It costs one forward solve per coefficient and
is meant for small meshes.
"""

from __future__ import annotations

import numpy as np

from .dg import ab3_coefficients, make_oracle
from .mesh import MeshGeometry, affine_factors
from .refelem import tet_basis

SOURCE_FIELDS = {"acoustic": (0,), "elastic": (3, 4, 5)}
RECEIVER_FIELDS = {"acoustic": (0,), "elastic": (0, 1, 2)}


def locate(elem_xyz: np.ndarray, x: np.ndarray, tol: float = 1e-12):
    """(element index, reference coordinates) of every point x (P, 3)."""
    F, _, _ = affine_factors(elem_xyz)
    Finv = np.linalg.inv(F)
    x = np.atleast_2d(np.asarray(x, dtype=float))
    ks = np.empty(len(x), dtype=np.int64)
    xis = np.empty((len(x), 3))
    for p, xp in enumerate(x):
        xi = np.einsum("kij,kj->ki", Finv, xp[None, :] - elem_xyz[:, 0, :]) - 1.0
        lam = np.concatenate([-(1.0 + xi.sum(1, keepdims=True)) / 2.0, (1.0 + xi) / 2.0], axis=1)
        inside = np.nonzero(np.all(lam >= -tol, axis=1))[0]
        if len(inside) == 0:
            raise ValueError(f"point {xp} is outside the mesh")
        ks[p] = inside[0]
        xis[p] = xi[inside[0]]
    return ks, xis


def lagrange_weights(ref, xi: np.ndarray) -> np.ndarray:
    """l(xi) (P, Np): u(xi) = l(xi) . u_nodes for u in the degree-N space."""
    xi = np.atleast_2d(xi)
    psi = tet_basis(ref.N, xi[:, 0], xi[:, 1], xi[:, 2])  # (P, Np)
    return np.linalg.solve(ref.V.T, psi.T).T


def ricker(t, f0: float, t0: float):
    a = (np.pi * f0 * (np.asarray(t, dtype=float) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


class MisfitProblem:
    """Forward solve with a point source and receivers, and the misfit."""

    def __init__(self, physics: str, mesh: MeshGeometry, elem_xyz: np.ndarray, dt: float, nsteps: int,
                 src_xyz, rec_xyz, f0: float, t0: float | None = None, absorbing=None):
        self.physics = physics
        self.mesh = mesh
        self.absorbing = absorbing  # optional (K, 4) mask of absorbing unpaired faces
        self.ref = mesh.ref
        self.dt = float(dt)
        self.nsteps = int(nsteps)
        self.f0 = float(f0)
        self.t0 = 1.2 / self.f0 if t0 is None else float(t0)
        self.nfields = 4 if physics == "acoustic" else 9
        ks, xis = locate(elem_xyz, np.atleast_2d(src_xyz))
        self.src_elem = ks
        self.src_weight = lagrange_weights(self.ref, xis)
        kr, xir = locate(elem_xyz, np.atleast_2d(rec_xyz))
        self.rec_elem = kr
        self.rec_weight = lagrange_weights(self.ref, xir)
        self.rec_fields = RECEIVER_FIELDS[physics]
        self.src_fields = SOURCE_FIELDS[physics]
        # b = (1/J_k) M^{-1} l(xi_s) in every source field
        K, Np = mesh.K, self.ref.Np
        self.b = np.zeros((K, self.nfields, Np))
        for k, w in zip(self.src_elem, self.src_weight):
            for c in self.src_fields:
                self.b[k, c] += (self.ref.Minv @ w) / mesh.J[k]
        self.wavelet = ricker(np.arange(self.nsteps + 1) * self.dt, self.f0, self.t0)

    @property
    def nchannels(self) -> int:
        return len(self.rec_elem) * len(self.rec_fields)

    def record(self, q: np.ndarray) -> np.ndarray:
        """Receiver values of one state, channel order (receiver, field)."""
        out = []
        for k, w in zip(self.rec_elem, self.rec_weight):
            for c in self.rec_fields:
                out.append(w @ q[k, c])
        return np.array(out)

    def forward(self, coef: np.ndarray) -> np.ndarray:
        """Receiver traces (nsteps + 1, channels) from the zero state; the
        arithmetic follows the coefficients' dtype (complex for the complex
        step)."""
        o = make_oracle(self.physics, self.mesh, coef, absorbing=self.absorbing)
        dtype = np.result_type(np.asarray(coef).dtype, float)
        q = np.zeros((self.mesh.K, self.nfields, self.ref.Np), dtype=dtype)
        traces = [self.record(q)]
        hist = []
        for m in range(self.nsteps):
            r = o.rhs(q) + self.wavelet[m] * self.b
            a = ab3_coefficients(m)
            upd = a[0] * r
            for i in (1, 2):
                if a[i] != 0.0:
                    upd = upd + a[i] * hist[-i]
            q = q + self.dt * upd
            hist = (hist + [r])[-2:]
            traces.append(self.record(q))
        return np.array(traces)

    def misfit(self, coef: np.ndarray, data: np.ndarray):
        u = self.forward(coef)
        res = u[1:] - data[1:]
        return 0.5 * self.dt * np.sum(res * res)

    def gradient_complex_step(self, coef: np.ndarray, data: np.ndarray, elems=None, h: float = 1e-30):
        """dJ/dcoef (K, ncoef); rows outside `elems` are left at zero."""
        coef = np.asarray(coef, dtype=float)
        K, nc = coef.shape
        grad = np.zeros((K, nc))
        for k in (range(K) if elems is None else elems):
            for p in range(nc):
                c = coef.astype(complex)
                c[k, p] += 1j * h
                grad[k, p] = np.imag(self.misfit(c, data)) / h
        return grad
