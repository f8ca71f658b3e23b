"""Affine geometry and face connectivity of a tetrahedral mesh (FP64 oracle).

Test infrastructure only.  The paper (Sec. 2.2, eq. (3)) uses per-element
volume factors g^vol_{k,i,j} and per-face surface factors g^sur_{k,f}, and a
per-face-node map to the neighbour's trace (Sec. 3.2).  Their definitions are
deferred to earlier work; the reading used here is the standard one for
affine tetrahedra:

* x(r,s,t) = x1 + F (r+1, s+1, t+1),  F = [x2-x1, x3-x1, x4-x1] / 2;
* J = det F (> 0),  G = F^{-T}, i.e. G[i, j] = d r_j / d x_i (this is g^vol);
* outward normal of face f: n_f = G nref_f / |G nref_f| with the
  unnormalised reference normals nref = (0,0,-1), (0,-1,0), (1,1,1), (-1,0,0),
  and Fscale_f = |G nref_f| = sJ_f / J (this is g^sur; sJ_f is the ratio of the
  physical face area to the area 2 of the parameter triangle).

Connectivity: faces pair up when they share the same three topological vertex
ids; face nodes pair up by matching physical coordinates (modulo the box
period for periodic meshes).  Unpaired faces are walls.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .refelem import FACE_VERTS, REF_FACE_NORMALS, RefElement, reference_element


@dataclass
class MeshGeometry:
    N: int
    K: int
    ref: RefElement
    xyz: np.ndarray  # (K, Np, 3) physical node coordinates
    J: np.ndarray  # (K,)
    G: np.ndarray  # (K, 3, 3)
    normals: np.ndarray  # (K, 4, 3)
    Fscale: np.ndarray  # (K, 4)
    EToE: np.ndarray  # (K, 4), -1 for a wall
    EToF: np.ndarray  # (K, 4), -1 for a wall
    nbr_node: np.ndarray  # (K, 4, Nfp) face-node index on the neighbour's face
    wall: np.ndarray  # (K, 4) bool


def affine_factors(elem_xyz: np.ndarray):
    """(F, J, G) for every element from its vertex coordinates."""
    x = np.asarray(elem_xyz, dtype=float)
    F = 0.5 * np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=-1)
    J = np.linalg.det(F)
    G = np.transpose(np.linalg.inv(F), (0, 2, 1))
    return F, J, G


def build_mesh(N: int, elem_xyz: np.ndarray, elem_topo: np.ndarray, period=None) -> MeshGeometry:
    ref = reference_element(N)
    elem_xyz = np.asarray(elem_xyz, dtype=float)
    elem_topo = np.asarray(elem_topo, dtype=np.int64)
    K = elem_xyz.shape[0]
    F, J, G = affine_factors(elem_xyz)
    if np.any(J <= 0.0):
        raise ValueError("element with non-positive Jacobian")
    rst1 = ref.r + 1.0  # (Np, 3)
    xyz = elem_xyz[:, None, 0, :] + np.einsum("kij,nj->kni", F, rst1)
    nvec = np.einsum("kij,fj->kfi", G, REF_FACE_NORMALS)
    Fscale = np.linalg.norm(nvec, axis=-1)
    normals = nvec / Fscale[..., None]

    # face pairing by topological vertex triples
    EToE = -np.ones((K, 4), dtype=np.int64)
    EToF = -np.ones((K, 4), dtype=np.int64)
    fv = np.array(FACE_VERTS)
    keys = np.sort(elem_topo[:, fv], axis=-1).reshape(K * 4, 3)
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    sk = keys[order]
    same = np.all(sk[1:] == sk[:-1], axis=1)
    if np.any(same[1:] & same[:-1]):
        raise ValueError("a face is shared by more than two elements")
    i1 = order[:-1][same]
    i2 = order[1:][same]
    EToE.reshape(-1)[i1] = i2 // 4
    EToF.reshape(-1)[i1] = i2 % 4
    EToE.reshape(-1)[i2] = i1 // 4
    EToF.reshape(-1)[i2] = i1 % 4
    wall = EToE < 0

    # face-node pairing by coordinates
    Nfp = ref.Nfp
    nbr_node = -np.ones((K, 4, Nfp), dtype=np.int64)
    xf = xyz[:, ref.Fmask, :]  # (K, 4, Nfp, 3)
    kk, ff = np.nonzero(~wall)
    per = None if period is None else np.asarray(period, dtype=float)
    chunk = 20000
    for s in range(0, len(kk), chunk):
        k1, f1 = kk[s : s + chunk], ff[s : s + chunk]
        k2, f2 = EToE[k1, f1], EToF[k1, f1]
        a = xf[k1, f1]  # (B, Nfp, 3)
        b = xf[k2, f2]
        d = a[:, :, None, :] - b[:, None, :, :]
        if per is not None:
            # axes with a zero period are not periodic
            d = d - per * np.round(d / np.where(per > 0.0, per, 1.0))
        dist = np.linalg.norm(d, axis=-1)  # (B, Nfp, Nfp)
        j = np.argmin(dist, axis=-1)
        if np.max(np.take_along_axis(dist, j[..., None], -1)) > 1e-9:
            raise ValueError("face nodes of neighbouring elements do not match")
        nbr_node[k1, f1] = j
    return MeshGeometry(
        N=N, K=K, ref=ref, xyz=xyz, J=J, G=G, normals=normals, Fscale=Fscale,
        EToE=EToE, EToF=EToF, nbr_node=nbr_node, wall=wall,
    )
