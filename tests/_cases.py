"""Shared builders for GPU-vs-oracle test cases.

Both sides are fed the same seeded inputs from ``dginputs`` (rounded to
float32, the precision the GPU path stores): mesh, coefficients and the
initial-data function, each side evaluating that function at its own node
coordinates.  Nothing here feeds a GPU result to the oracle.
"""

from __future__ import annotations

import sys

import numpy as np

import dginputs as di
from oracle.dg import make_oracle
from oracle.mesh import build_mesh


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def coefficients(physics: str, mesh, kind: str, seed: int = 1) -> np.ndarray:
    if physics == "acoustic":
        if kind == "constant":
            c = di.acoustic_constant(mesh)
        elif kind == "layers":
            c = di.acoustic_two_layer(mesh)
        else:
            c = di.acoustic_loguniform(mesh, seed)
    elif physics == "anisotropic":
        if kind == "constant":
            c = di.anisotropic_from_isotropic(di.elastic_constant(mesh))
        else:
            c = di.anisotropic_random(mesh, seed)
    else:
        if kind == "constant":
            c = di.elastic_constant(mesh)
        else:
            c = di.elastic_loguniform(mesh, seed)
    return c.astype(np.float32).astype(np.float64)


def initial_fields(physics: str, xyz: np.ndarray, kind: str = "gaussian") -> np.ndarray:
    """[K, Nf, Np] from node coordinates [K, Np, 3]."""
    if kind == "gaussian":
        f = di.acoustic_gaussian(xyz) if physics == "acoustic" else di.elastic_gaussian(xyz)
    elif kind == "pulses":
        f = di.gaussian_pulses(xyz, 4 if physics == "acoustic" else 9)
    elif kind == "smooth":
        # a smooth state that excites every field (all non-zero)
        nf = 4 if physics == "acoustic" else 9
        f = np.stack(
            [np.sin(2.0 + c + 3.1 * xyz[..., 0] - 1.7 * xyz[..., 1] + (0.5 + 0.3 * c) * xyz[..., 2]) for c in range(nf)]
        )
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(np.moveaxis(f, 0, 1)).astype(np.float32).astype(np.float64)


class Case:
    """One mesh / physics / degree, set up on both the GPU and the oracle."""

    def __init__(self, physics, N, n, jitter=0.1, seed=0, coef_kind="random", periodic=False,
                 init="gaussian", dims=None, mesh=None, absorbing=None):
        """``absorbing``: None (reflecting walls), "all" or "half" (a seeded
        random half of the unpaired faces absorb), or a (K, 4) bool mask."""
        import torch

        from paper_1602_07997_amd import DGSolver

        self.physics, self.N = physics, N
        if mesh is None:
            dims = dims or (n, n, n)
            mesh = di.kuhn_box(*dims, jitter=jitter, seed=seed, periodic=periodic)
        self.mesh = mesh
        self.coef = coefficients(physics, mesh, coef_kind, seed + 1)
        self.solver = DGSolver(physics, N, mesh.elem_xyz, mesh.elem_topo)
        self.solver.set_coefficients(torch.tensor(self.coef, dtype=torch.float32, device="cuda"))
        self.q0_gpu = initial_fields(physics, self.solver.node_coordinates(), init)
        self.geo = build_mesh(N, mesh.elem_xyz, mesh.elem_topo, mesh.period)
        if isinstance(absorbing, str):
            if absorbing == "all":
                absorbing = self.geo.wall.copy()
            else:
                absorbing = self.geo.wall & (np.random.default_rng(seed + 99).random(self.geo.wall.shape) < 0.5)
        self.absorbing = absorbing
        if absorbing is not None:
            self.solver.set_boundary(absorbing)
        self.oracle = make_oracle(physics, self.geo, self.coef, absorbing=absorbing)
        self.q0 = initial_fields(physics, self.geo.xyz, init)
        self.dt = di.time_step(mesh, N, di.max_wave_speed(self.coef, physics))

    def to_gpu(self, a):
        import torch

        return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda").contiguous()

    @staticmethod
    def to_host(t) -> np.ndarray:
        return t.detach().cpu().numpy().astype(np.float64)

    def rel_l2(self, q_gpu: np.ndarray, q_ref: np.ndarray):
        return self.oracle.rel_l2(q_gpu, q_ref)

    def check(self, q_gpu: np.ndarray, q_ref: np.ndarray, l2: float, what: str = "", per_field: float | None = None,
              node: float | None = None):
        """Asserts the GPU result against the oracle's, see ``check_close``."""
        return check_close(self.oracle, q_gpu, q_ref, l2, what, per_field, node)


def node_errors(q: np.ndarray, q_ref: np.ndarray) -> np.ndarray:
    """Element-wise error per field: max over elements and nodes of |q - q_ref|
    divided by the field's largest |q_ref| (floored at 1e-3 of the largest
    field maximum, so that a field that is nearly zero is measured against
    the state's scale)."""
    d = np.abs(q - q_ref).max(axis=(0, 2))
    scale = np.abs(q_ref).max(axis=(0, 2))
    return d / np.maximum(scale, 1e-3 * scale.max())


def check_close(oracle, q: np.ndarray, q_ref: np.ndarray, l2: float, what: str = "",
                per_field: float | None = None, node: float | None = None):
    """Mass-weighted relative L2 over all fields <= l2, per field <=
    per_field (default l2) and, node by node, |q - q_ref| <= node times the
    field's largest |q_ref| (default 10 l2).  The node-wise bar catches a
    single wrong element that the norms would average away.  Returns
    (overall L2, per-field L2, per-field node-wise ratio)."""
    per_field = l2 if per_field is None else per_field
    node = 10.0 * l2 if node is None else node
    err, per = oracle.rel_l2(q, q_ref)
    nd = node_errors(q, q_ref)
    log(f"  {what} rel L2 {err:.2e}, per field max {np.nanmax(per):.2e}, node-wise max {nd.max():.2e}")
    assert err <= l2, (what, err)
    assert np.all(np.nan_to_num(per) <= per_field), (what, per)
    assert np.all(nd <= node), (what, nd)
    return err, per, nd
