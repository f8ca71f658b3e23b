"""Right-hand sides, Adams-Bashforth update and energy (FP64 oracle).

Test infrastructure only.  Everything is the plain definition, vectorised over
elements with NumPy; no blocking, fusion or reordering beyond the formulas.

Acoustic system (Sec. 2.1; eqs. (5)-(6)), fields (p, v1, v2, v3):
  r^p   = -rho c^2 sum_j D_j [sum_i g_ij v_i] - L (Fscale p_p)
  r^v_i = -(1/rho) sum_j g_ij D_j p            - L (Fscale p_v n_i)
  p_p = -(rho c^2)^- k_c alpha,  p_v = c^- k_c alpha,
  alpha = [[p]] - (rho c)^+ [[v_n]],  k_c = 1/{rho c},
  [[p]] = (p^+ - p^-)/2,  [[v_n]] = (v^+ - v^-).n/2,  {a} = (a^- + a^+)/2.

Isotropic elastic system (Sec. 2.1 and the elastic right-hand side of
Sec. 3.2), fields (v1, v2, v3, s11, s22, s33, s23, s13, s12):
  r^v_i    = (1/rho) sum_n D_n [sum_m g_mn s_im] + L (Fscale p_v)_i
  r^s_ij   = delta_ij lambda div v + mu (d v_i/d x_j + d v_j/d x_i)
             + L (Fscale P_s)_ij
  The paper prints the mu term with garbled indices; the reading used is
  mu sum_n (g_jn D_n v_i + g_in D_n v_j), i.e. 2 mu sym(grad v) as in the PDE.
  P_s = k_p a_p lambda^- I + 2 (k_p a_p - k_s a_s) mu^- n n^T
        + k_s mu^- (n a_s^T + a_s n^T)
  p_v = (k_p a_p c_p^- - k_s a_s c_s^-) n + k_s c_s^- a_s(vector),
  a_p = [[s_nn]] + (rho c_p)^+ [[v_n]],  a_s = [[s_nn]] + (rho c_s)^+ [[v_n]],
  a_s(vector) = [[s n]] + (rho c_s)^+ [[v]],  k_p = 1/{rho c_p},
  k_s = 1/{rho c_s}, jumps halved as above, n the outward normal of the
  element ("-" side).

Walls (unpaired faces; the paper is silent): mirror ghost state with the
element's own coefficients -- acoustic p^+ = p^-, v_n^+ = -v_n^- (rigid wall);
elastic v^+ = v^-, (s n)^+ = -(s n)^- (traction-free).

Anisotropic elastic system (Sec. 5 names anisotropic media as future work;
the reading is ours), the elastic fields with a general symmetric positive
definite Voigt stiffness C per element: volume terms as above with C e(v) in
place of lambda div v I + 2 mu sym(grad v), and the Riemann solution of a
medium whose waves all travel with one impedance Z = sqrt(rho max_a C_aa)
per side (see AnisotropicElasticOracle).

Absorbing faces (an optional subset of the unpaired faces; Sec. 5 names
artificial boundary conditions as future work, so the reading is ours): the
exterior state is zero, with the element's own coefficients.  The upwind
flux of Sec. 2.1 then solves the Riemann problem against a medium at rest,
so no characteristic enters through the face: acoustic alpha reduces to
-(p - Z v_n)^-/2, the element's own incoming characteristic.

Time stepping (eq. (4)): q^{m+1} = q^m + dt (a1 r^m + a2 r^{m-1} + a3 r^{m-2}),
a = (23, -16, 5)/12.  The paper is silent on the start: step 0 uses forward
Euler, step 1 the two-step formula (3/2, -1/2), unless the history is given.
"""

from __future__ import annotations

import numpy as np

from .mesh import MeshGeometry

# Voigt order of the stress components and the full-tensor lookup
VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
TENSOR_INDEX = np.array([[0, 5, 4], [5, 1, 3], [4, 3, 2]])


def ab3_coefficients(m: int):
    """Adams-Bashforth weights for step m with the start-up reading."""
    if m == 0:
        return (1.0, 0.0, 0.0)
    if m == 1:
        return (1.5, -0.5, 0.0)
    return (23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0)


class _Base:
    nfields = 0

    def __init__(self, mesh: MeshGeometry, coef: np.ndarray, absorbing=None):
        self.mesh = mesh
        self.ref = mesh.ref
        # real coefficients in float64; complex ones are kept (complex-step
        # derivatives of functions of the coefficients)
        self.coef = np.asarray(coef)
        if not np.iscomplexobj(self.coef):
            self.coef = self.coef.astype(float)
        if self.coef.shape != (mesh.K, self.ncoef):
            raise ValueError("coefficient array has the wrong shape")
        self.K = mesh.K
        if absorbing is None:
            absorbing = np.zeros((mesh.K, 4), dtype=bool)
        self.absorbing = np.asarray(absorbing, dtype=bool)
        if self.absorbing.shape != (mesh.K, 4) or np.any(self.absorbing & ~mesh.wall):
            raise ValueError("absorbing faces must be a (K, 4) mask of unpaired faces")
        # neighbour lookups for every face node (walls point to themselves)
        K, Nfp = mesh.K, self.ref.Nfp
        kk = np.repeat(np.arange(K)[:, None], 4, axis=1)
        ff = np.repeat(np.arange(4)[None, :], K, axis=0)
        self.nb_elem = np.where(mesh.wall, kk, mesh.EToE)
        nb_face = np.where(mesh.wall, ff, mesh.EToF)
        nb_node = np.where(mesh.wall[..., None], np.arange(Nfp)[None, None, :], mesh.nbr_node)
        # volume node index on the neighbour for each own face node
        self.nb_vol = self.ref.Fmask[nb_face[..., None], nb_node]  # (K, 4, Nfp)
        self.nb_el3 = np.broadcast_to(self.nb_elem[..., None], (K, 4, Nfp))

    # helpers ---------------------------------------------------------------
    def ref_derivs(self, u: np.ndarray) -> np.ndarray:
        """u (..., Np) -> (..., 3, Np) with [..., j, :] = D_j u."""
        return np.stack([u @ self.ref.D[j].T for j in range(3)], axis=-2)

    def lift(self, flux: np.ndarray) -> np.ndarray:
        """flux (K, ..., 4, Nfp) -> (K, ..., Np) = LIFT @ flux."""
        sh = flux.shape
        return flux.reshape(sh[:-2] + (4 * sh[-1],)) @ self.ref.LIFT.T

    def own_face(self, u: np.ndarray) -> np.ndarray:
        """u (K, Np) -> (K, 4, Nfp)."""
        return u[:, self.ref.Fmask]

    def nbr_face(self, u: np.ndarray) -> np.ndarray:
        """u (K, Np) -> neighbour values at each own face node (K, 4, Nfp)."""
        return u[self.nb_el3, self.nb_vol]

    def mass_norm2(self, u: np.ndarray) -> np.ndarray:
        """Per element J_k u^T M u for u (K, Np)."""
        return self.mesh.J * np.einsum("kn,nm,km->k", u, self.ref.M, u)

    def rel_l2(self, q: np.ndarray, q_ref: np.ndarray):
        """Mass-weighted relative L2 error (overall, per field) of q vs q_ref."""
        e = q - q_ref
        num = np.array([self.mass_norm2(e[:, c]).sum() for c in range(self.nfields)])
        den = np.array([self.mass_norm2(q_ref[:, c]).sum() for c in range(self.nfields)])
        overall = float(np.sqrt(num.sum() / den.sum()))
        with np.errstate(divide="ignore", invalid="ignore"):
            per = np.sqrt(num / np.where(den > 0, den, np.nan))
        return overall, per


class AcousticOracle(_Base):
    nfields = 4
    ncoef = 2  # (rho, c)

    def __init__(self, mesh, coef, absorbing=None):
        super().__init__(mesh, coef, absorbing)
        rho, c = self.coef[:, 0], self.coef[:, 1]
        self.rho, self.c = rho, c
        self.Z = rho * c
        self.Znb = np.where(self.mesh.wall, self.Z[:, None], self.Z[self.nb_elem])

    def rhs(self, q: np.ndarray) -> np.ndarray:
        mesh = self.mesh
        G = mesh.G
        p, v = q[:, 0], q[:, 1:4]
        rho, c = self.rho, self.c
        # volume terms
        Dp = self.ref_derivs(p)  # (K, 3, Np)
        grad_p = np.einsum("kij,kjn->kin", G, Dp)
        Dv = self.ref_derivs(v)  # (K, 3(i), 3(j), Np)
        div_v = np.einsum("kij,kijn->kn", G, Dv)
        r = np.empty_like(q)
        r[:, 0] = -(rho * c * c)[:, None] * div_v
        r[:, 1:4] = -(1.0 / rho)[:, None, None] * grad_p
        # surface terms
        n = mesh.normals  # (K, 4, 3)
        pM = self.own_face(p)
        vnM = np.einsum("kfi,kifj->kfj", n, v[:, :, mesh.ref.Fmask])
        pP = self.nbr_face(p)
        vP = np.stack([self.nbr_face(v[:, i]) for i in range(3)], axis=1)
        vnP = np.einsum("kfi,kifj->kfj", n, vP)
        wall = mesh.wall[..., None]
        pP = np.where(wall, pM, pP)
        vnP = np.where(wall, -vnM, vnP)
        absorb = self.absorbing[..., None]
        pP = np.where(absorb, 0.0, pP)
        vnP = np.where(absorb, 0.0, vnP)
        Zm = self.Z[:, None, None]
        Zp = self.Znb[..., None]
        jp = 0.5 * (pP - pM)
        jv = 0.5 * (vnP - vnM)
        kc = 2.0 / (Zm + Zp)
        alpha = jp - Zp * jv
        Fs = mesh.Fscale[..., None]
        flux_p = Fs * (rho * c * c)[:, None, None] * kc * alpha
        r[:, 0] += self.lift(flux_p)
        base = -Fs * c[:, None, None] * kc * alpha  # (K, 4, Nfp)
        for i in range(3):
            r[:, 1 + i] += self.lift(base * n[:, :, i][..., None])
        return r

    def energy_density(self, q: np.ndarray) -> np.ndarray:
        """Per element 1/2 J_k (p^T M p/(rho c^2) + rho sum v_i^T M v_i)."""
        e = self.mass_norm2(q[:, 0]) / (self.rho * self.c**2)
        for i in range(3):
            e = e + self.rho * self.mass_norm2(q[:, 1 + i])
        return 0.5 * e

    def energy(self, q: np.ndarray) -> float:
        return float(self.energy_density(q).sum())

    def energy_rate(self, q: np.ndarray) -> float:
        """dE/dt = sum_k J_k (p^T M r_p/(rho c^2) + rho sum v_i^T M r_vi)."""
        r = self.rhs(q)
        M, J = self.ref.M, self.mesh.J
        w = np.concatenate([(1.0 / (self.rho * self.c**2))[:, None], np.repeat(self.rho[:, None], 3, 1)], 1)
        return float(np.einsum("k,kc,kcn,nm,kcm->", J, w, q, M, r))


class ElasticOracle(_Base):
    nfields = 9
    ncoef = 3  # (rho, lambda, mu)

    def __init__(self, mesh, coef, absorbing=None):
        super().__init__(mesh, coef, absorbing)
        rho, lam, mu = self.coef[:, 0], self.coef[:, 1], self.coef[:, 2]
        if np.any(np.real(mu) <= 0.0):
            raise ValueError("the elastic flux needs mu > 0")
        self.rho, self.lam, self.mu = rho, lam, mu
        self.cp = np.sqrt((lam + 2.0 * mu) / rho)
        self.cs = np.sqrt(mu / rho)
        self.Zp = rho * self.cp
        self.Zs = rho * self.cs
        w = self.mesh.wall
        self.Zp_nb = np.where(w, self.Zp[:, None], self.Zp[self.nb_elem])
        self.Zs_nb = np.where(w, self.Zs[:, None], self.Zs[self.nb_elem])

    @staticmethod
    def tensor(s: np.ndarray) -> np.ndarray:
        """Voigt (K, 6, ...) -> full (K, 3, 3, ...)."""
        return s[:, TENSOR_INDEX]

    def rhs(self, q: np.ndarray) -> np.ndarray:
        mesh = self.mesh
        G = mesh.G
        v = q[:, 0:3]
        S = self.tensor(q[:, 3:9])  # (K, 3, 3, Np)
        rho, lam, mu = self.rho, self.lam, self.mu
        # volume terms
        Dv = self.ref_derivs(v)  # (K, 3 i, 3 l, Np): D_l v_i
        grad_v = np.einsum("kjl,kiln->kijn", G, Dv)  # d v_i / d x_j
        div_v = np.einsum("kiin->kn", grad_v)
        DS = self.ref_derivs(q[:, 3:9])  # (K, 6, 3 l, Np)
        DS = DS[:, TENSOR_INDEX]  # (K, 3 i, 3 j, 3 l, Np)
        div_s = np.einsum("kjl,kijln->kin", G, DS, optimize=True)  # sum_j d s_ij / d x_j
        r = np.empty_like(q)
        r[:, 0:3] = (1.0 / rho)[:, None, None] * div_s
        for a, (i, j) in enumerate(VOIGT):
            val = mu[:, None] * (grad_v[:, i, j] + grad_v[:, j, i])
            if i == j:
                val = val + lam[:, None] * div_v
            r[:, 3 + a] = val
        # surface terms
        n = mesh.normals  # (K, 4, 3)
        Fm = mesh.ref.Fmask
        vM = v[:, :, Fm]  # (K, 3, 4, Nfp)
        SM = S[:, :, :, Fm]  # (K, 3, 3, 4, Nfp)
        vP = np.stack([self.nbr_face(v[:, i]) for i in range(3)], axis=1)
        sP = np.stack([self.nbr_face(q[:, 3 + a]) for a in range(6)], axis=1)
        SP = self.tensor(sP)
        tM = np.einsum("kijfx,kfj->kifx", SM, n)  # (s^- n)_i
        tP = np.einsum("kijfx,kfj->kifx", SP, n)  # (s^+ n)_i, own normal
        wall = mesh.wall[None, :, :, None].transpose(1, 0, 2, 3)  # (K,1,4,1)
        vP = np.where(wall, vM, vP)
        tP = np.where(wall, -tM, tP)
        absorb = self.absorbing[:, None, :, None]
        vP = np.where(absorb, 0.0, vP)
        tP = np.where(absorb, 0.0, tP)
        jv = 0.5 * (vP - vM)  # (K, 3, 4, Nfp)
        jt = 0.5 * (tP - tM)
        jvn = np.einsum("kifx,kfi->kfx", jv, n)
        jsnn = np.einsum("kifx,kfi->kfx", jt, n)
        Zpm, Zsm = self.Zp[:, None, None], self.Zs[:, None, None]
        Zpp, Zsp = self.Zp_nb[..., None], self.Zs_nb[..., None]
        kp = 2.0 / (Zpm + Zpp)
        ks = 2.0 / (Zsm + Zsp)
        ap = jsnn + Zpp * jvn
        as_ = jsnn + Zsp * jvn
        asv = jt + Zsp[:, None] * jv  # (K, 3, 4, Nfp)
        lam3, mu3 = lam[:, None, None], mu[:, None, None]
        cp3, cs3 = self.cp[:, None, None], self.cs[:, None, None]
        Fs = mesh.Fscale[..., None]
        nn = n.transpose(0, 2, 1)[..., None]  # (K, 3, 4, 1)
        # velocity penalty
        pv = (kp * ap * cp3 - ks * as_ * cs3)[:, None] * nn + (ks * cs3)[:, None] * asv
        r[:, 0:3] += self.lift(Fs[:, None] * pv)
        # stress penalty
        A = kp * ap * lam3
        B = 2.0 * (kp * ap - ks * as_) * mu3
        C = ks * mu3
        for a, (i, j) in enumerate(VOIGT):
            Ps = B * nn[:, i] * nn[:, j] + C * (nn[:, i] * asv[:, j] + asv[:, i] * nn[:, j])
            if i == j:
                Ps = Ps + A
            r[:, 3 + a] += self.lift(Fs * Ps)
        return r

    def energy_density(self, q: np.ndarray) -> np.ndarray:
        """Per element 1/2 J_k [rho |v|^2 + (1/(2mu))(s:s - lam/(3lam+2mu) tr(s)^2)]
        integrated with the mass matrix (off-diagonal stresses count twice)."""
        rho, lam, mu = self.rho, self.lam, self.mu
        e = np.zeros(self.K)
        for i in range(3):
            e += rho * self.mass_norm2(q[:, i])
        ss = np.zeros(self.K)
        for a, (i, j) in enumerate(VOIGT):
            ss += (1.0 if i == j else 2.0) * self.mass_norm2(q[:, 3 + a])
        tr = q[:, 3] + q[:, 4] + q[:, 5]
        e += (ss - lam / (3.0 * lam + 2.0 * mu) * self.mass_norm2(tr)) / (2.0 * mu)
        return 0.5 * e

    def energy(self, q: np.ndarray) -> float:
        return float(self.energy_density(q).sum())

    def energy_rate(self, q: np.ndarray) -> float:
        """Semi-discrete dE/dt = <q, r>_E (the energy inner product of q and r)."""
        r = self.rhs(q)
        rho, lam, mu = self.rho, self.lam, self.mu
        J, M = self.mesh.J, self.ref.M

        def ip(a, b):
            return J * np.einsum("kn,nm,km->k", a, M, b)

        e = np.zeros(self.K)
        for i in range(3):
            e += rho * ip(q[:, i], r[:, i])
        ss = np.zeros(self.K)
        for a, (i, j) in enumerate(VOIGT):
            ss += (1.0 if i == j else 2.0) * ip(q[:, 3 + a], r[:, 3 + a])
        trq = q[:, 3] + q[:, 4] + q[:, 5]
        trr = r[:, 3] + r[:, 4] + r[:, 5]
        e += (ss - lam / (3.0 * lam + 2.0 * mu) * ip(trq, trr)) / (2.0 * mu)
        return float(e.sum())


# Upper triangle of the 6x6 Voigt stiffness, row by row: the order of the 21
# stiffness coefficients after rho in an anisotropic coefficient row.
UPPER6 = [(a, b) for a in range(6) for b in range(a, 6)]


def stiffness_matrix(c21: np.ndarray) -> np.ndarray:
    """(..., 21) upper-triangle entries -> (..., 6, 6) symmetric Voigt C."""
    c21 = np.asarray(c21)
    C = np.zeros(c21.shape[:-1] + (6, 6), dtype=c21.dtype)
    for i, (a, b) in enumerate(UPPER6):
        C[..., a, b] = c21[..., i]
        C[..., b, a] = c21[..., i]
    return C


class AnisotropicElasticOracle(_Base):
    """Linear elasticity with a general stiffness per element (an extension
    the paper names as future work, Sec. 5; the reading is ours):

      rho dv/dt = div s,   ds/dt = C e(v)

    with Voigt s = (s11, s22, s33, s23, s13, s12), engineering strain
    e = (e11, e22, e33, 2 e23, 2 e13, 2 e12) and C symmetric positive definite
    (21 coefficients).  Volume terms as in the elastic right-hand side of
    Sec. 3.2 with C in place of lambda, mu.  Surface: the Riemann solution of
    a medium whose waves all travel with one impedance Z per side (the
    acoustic-like solution applied to every traction / velocity component),
      t* = (Z+ t- + Z- t+)/(Z- + Z+) + Z- Z+/(Z- + Z+) (v+ - v-),
      v* = (Z- v- + Z+ v+)/(Z- + Z+) + (t+ - t-)/(Z- + Z+),
    t = s n with the own normal n, entering as the strong-form corrections
      r_v += LIFT((t* - t-)/rho),   r_s += LIFT(C e(n (x) (v* - v-))),
    with Z = sqrt(rho max_a C_aa) (for an isotropic C, max C_aa = lambda + 2 mu
    and Z is the P impedance).  Per face the energy then changes by
    -(Z- Z+/(Z- + Z+)) |[v]|^2 - |[t]|^2/(Z- + Z+) <= 0 for any Z > 0.
    Walls: traction-free mirror state (t+ = -t-, v+ = v-, Z+ = Z-); absorbing
    faces: zero exterior state.

    Coefficients per element: (rho, then the 21 upper-triangle entries of C
    in the row order of UPPER6).
    """

    nfields = 9
    ncoef = 22

    def __init__(self, mesh, coef, absorbing=None):
        super().__init__(mesh, coef, absorbing)
        self.rho = self.coef[:, 0]
        self.C = stiffness_matrix(self.coef[:, 1:])
        diag = np.stack([self.C[:, a, a] for a in range(6)], axis=1)
        # largest diagonal stiffness (chosen on the real part, so that a
        # complex-step perturbation keeps the same entry)
        self.Z = np.sqrt(self.rho * diag[np.arange(self.K), np.argmax(np.real(diag), axis=1)])
        w = self.mesh.wall
        self.Znb = np.where(w, self.Z[:, None], self.Z[self.nb_elem])

    @staticmethod
    def strain_voigt(grad_v):
        """grad_v (..., 3 i, 3 j, ...) = d v_i / d x_j -> engineering strain (..., 6, ...)."""
        g = grad_v
        return np.stack([g[:, 0, 0], g[:, 1, 1], g[:, 2, 2], g[:, 1, 2] + g[:, 2, 1],
                         g[:, 0, 2] + g[:, 2, 0], g[:, 0, 1] + g[:, 1, 0]], axis=1)

    def rhs(self, q: np.ndarray) -> np.ndarray:
        mesh = self.mesh
        G = mesh.G
        v = q[:, 0:3]
        rho = self.rho
        Dv = self.ref_derivs(v)  # (K, 3 i, 3 l, Np)
        grad_v = np.einsum("kjl,kiln->kijn", G, Dv)  # d v_i / d x_j
        DS = self.ref_derivs(q[:, 3:9])[:, TENSOR_INDEX]  # (K, 3 i, 3 j, 3 l, Np)
        div_s = np.einsum("kjl,kijln->kin", G, DS, optimize=True)
        r = np.empty_like(q)
        r[:, 0:3] = (1.0 / rho)[:, None, None] * div_s
        r[:, 3:9] = np.einsum("kab,kbn->kan", self.C, self.strain_voigt(grad_v))
        # surface terms
        n = mesh.normals  # (K, 4, 3)
        Fm = mesh.ref.Fmask
        vM = v[:, :, Fm]  # (K, 3, 4, Nfp)
        SM = ElasticOracle.tensor(q[:, 3:9])[:, :, :, Fm]
        vP = np.stack([self.nbr_face(v[:, i]) for i in range(3)], axis=1)
        SP = ElasticOracle.tensor(np.stack([self.nbr_face(q[:, 3 + a]) for a in range(6)], axis=1))
        tM = np.einsum("kijfx,kfj->kifx", SM, n)
        tP = np.einsum("kijfx,kfj->kifx", SP, n)
        wall = mesh.wall[:, None, :, None]
        vP = np.where(wall, vM, vP)
        tP = np.where(wall, -tM, tP)
        absorb = self.absorbing[:, None, :, None]
        vP = np.where(absorb, 0.0, vP)
        tP = np.where(absorb, 0.0, tP)
        Zm = self.Z[:, None, None, None]
        Zp = self.Znb[:, None, :, None]
        S = Zm + Zp
        t_star = (Zp * tM + Zm * tP) / S + (Zm * Zp / S) * (vP - vM)
        v_star = (Zm * vM + Zp * vP) / S + (tP - tM) / S
        Fs = mesh.Fscale[:, None, :, None]
        r[:, 0:3] += self.lift(Fs * (t_star - tM) / rho[:, None, None, None])
        w_ = Fs * (v_star - vM)  # (K, 3, 4, Nfp)
        nn = n.transpose(0, 2, 1)[..., None]  # (K, 3, 4, 1)
        ew = np.stack([nn[:, 0] * w_[:, 0], nn[:, 1] * w_[:, 1], nn[:, 2] * w_[:, 2],
                       nn[:, 1] * w_[:, 2] + nn[:, 2] * w_[:, 1], nn[:, 0] * w_[:, 2] + nn[:, 2] * w_[:, 0],
                       nn[:, 0] * w_[:, 1] + nn[:, 1] * w_[:, 0]], axis=1)  # (K, 6, 4, Nfp)
        r[:, 3:9] += self.lift(np.einsum("kab,kbfx->kafx", self.C, ew))
        return r

    def _compliance(self):
        return np.linalg.inv(self.C)

    def energy_density(self, q: np.ndarray) -> np.ndarray:
        """Per element 1/2 J_k [rho |v|^2 + s^T C^-1 s] with the mass matrix."""
        e = np.zeros(self.K, dtype=np.result_type(q, self.coef))
        for i in range(3):
            e = e + self.rho * self.mass_norm2(q[:, i])
        Sc = self._compliance()
        J, M = self.mesh.J, self.ref.M
        e = e + J * np.einsum("kan,nm,kab,kbm->k", q[:, 3:9], M, Sc, q[:, 3:9])
        return 0.5 * e

    def energy(self, q: np.ndarray) -> float:
        return float(np.real(self.energy_density(q).sum()))

    def energy_rate(self, q: np.ndarray) -> float:
        r = self.rhs(q)
        J, M = self.mesh.J, self.ref.M
        e = np.einsum("k,kin,nm,kim->k", J * self.rho, q[:, 0:3], M, r[:, 0:3])
        e = e + J * np.einsum("kan,nm,kab,kbm->k", q[:, 3:9], M, self._compliance(), r[:, 3:9])
        return float(e.sum())


def make_oracle(physics: str, mesh: MeshGeometry, coef: np.ndarray, absorbing=None):
    """``absorbing``: optional (K, 4) bool mask of unpaired faces that absorb
    instead of reflecting."""
    if physics == "acoustic":
        return AcousticOracle(mesh, coef, absorbing)
    if physics == "elastic":
        return ElasticOracle(mesh, coef, absorbing)
    if physics == "anisotropic":
        return AnisotropicElasticOracle(mesh, coef, absorbing)
    raise ValueError(physics)


class AB3Stepper:
    """Third-order Adams-Bashforth time loop (eq. (4)) over an oracle's RHS.

    ``source(m, t)`` optionally returns an additive forcing for r^m.
    """

    def __init__(self, oracle, q0: np.ndarray, history=None, step_index: int = 0):
        self.oracle = oracle
        self.q = np.array(q0, copy=True)
        if not np.issubdtype(self.q.dtype, np.inexact):
            self.q = self.q.astype(float)
        self.r1 = None if history is None else np.array(history[0], dtype=float)
        self.r2 = None if history is None else np.array(history[1], dtype=float)
        self.m = step_index

    def step(self, nsteps: int, dt: float):
        for _ in range(nsteps):
            r0 = self.oracle.rhs(self.q)
            a1, a2, a3 = ab3_coefficients(self.m)
            upd = a1 * r0
            if a2 != 0.0:
                upd = upd + a2 * self.r1
            if a3 != 0.0:
                upd = upd + a3 * self.r2
            self.q = self.q + dt * upd
            self.r2, self.r1 = self.r1, r0
            self.m += 1
        return self.q
