"""Python front end of the dgwave C ABI.

Marshals numpy / torch arrays into the C calls; every step of the hot path
runs in the library's HIP kernels.  Torch supplies the device memory (one
uint8 workspace per solver, batch and misfit, sized by the library's
*_workspace_bytes queries) and the stream; the library allocates none.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as nat
from ._native import check, lib

PHYSICS = {"acoustic": nat.DG_ACOUSTIC, "elastic": nat.DG_ELASTIC, "anisotropic": nat.DG_ANISOTROPIC}
NCOEF = {"acoustic": 2, "elastic": 3, "anisotropic": 22}  # rho, c | rho, lambda, mu | rho, 21 stiffness entries


def ref_sizes(order: int):
    Np, Nfp = C.c_int(), C.c_int()
    check(lib.dg_ref_sizes(order, C.byref(Np), C.byref(Nfp)), "dg_ref_sizes")
    return Np.value, Nfp.value


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i32ptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _i64ptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def reference_operators(order: int) -> dict:
    """Host-side reference element of the product (no GPU needed)."""
    Np, Nfp = ref_sizes(order)
    nodes = np.zeros((Np, 3))
    D = np.zeros((3, Np, Np))
    mass = np.zeros((Np, Np))
    lift = np.zeros((Np, 4 * Nfp))
    fmask = np.zeros((4, Nfp), dtype=np.int32)
    check(
        lib.dg_reference_operators(order, _dptr(nodes), _dptr(D), _dptr(mass), _dptr(lift), _i32ptr(fmask)),
        "dg_reference_operators",
    )
    perm = np.zeros((6, Nfp), dtype=np.int32)
    check(lib.dg_face_permutations(order, _i32ptr(perm)), "dg_face_permutations")
    return {"nodes": nodes, "D": D, "mass": mass, "lift": lift, "fmask": fmask, "perm": perm}


def mesh_connectivity(elem_topo: np.ndarray):
    topo = np.ascontiguousarray(elem_topo, dtype=np.int64)
    K = topo.shape[0]
    e2e = np.zeros((K, 4), dtype=np.int64)
    e2f = np.zeros((K, 4), dtype=np.int32)
    orient = np.zeros((K, 4), dtype=np.int32)
    check(lib.dg_mesh_connectivity(K, _i64ptr(topo), _i64ptr(e2e), _i32ptr(e2f), _i32ptr(orient)), "dg_mesh_connectivity")
    return e2e, e2f, orient


def _require_torch_device_tensor(t, shape, name):
    """Validates a device float32 tensor of the given shape; returns its pointer."""
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


class DGSolver:
    """One mesh, one degree, one physics on the current GPU.

    ``elem_xyz`` float64 [K,4,3] and ``elem_topo`` int64 [K,4] (host numpy).
    Field tensors are torch float32 [K, Nfields, Np] on the GPU.
    """

    def __init__(self, physics: str, order: int, elem_xyz, elem_topo, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("DGSolver needs a GPU")
        self.physics = physics
        self.order = order
        self.xyz = np.ascontiguousarray(elem_xyz, dtype=np.float64)
        self.topo = np.ascontiguousarray(elem_topo, dtype=np.int64)
        self.K = int(self.xyz.shape[0])
        self.Np, self.Nfp = ref_sizes(order)
        self.nfields = lib.dg_num_fields(PHYSICS[physics])
        self.ncoef = NCOEF[physics]
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        # every device array of the solver lives in one torch-owned buffer
        nbytes = C.c_size_t(0)
        check(lib.dg_workspace_bytes(PHYSICS[physics], order, self.K, C.byref(nbytes)), "dg_workspace_bytes")
        with torch.cuda.stream(stream):
            self._workspace = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        check(
            lib.dg_create(
                PHYSICS[physics], order, self.K, _dptr(self.xyz), _i64ptr(self.topo),
                C.c_void_p(self._workspace.data_ptr()), nbytes, C.c_void_p(stream.cuda_stream), C.byref(h),
            ),
            "dg_create",
        )
        self._h = h

    @property
    def workspace_bytes(self) -> int:
        return int(self._workspace.numel())

    # lifecycle ---------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib.dg_destroy(self._h)
            self._h = None
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes ------------------------------------------------------------------
    @property
    def field_shape(self):
        return (self.K, self.nfields, self.Np)

    def empty_fields(self):
        import torch

        return torch.empty(self.field_shape, dtype=torch.float32, device="cuda")

    # calls -------------------------------------------------------------------
    def node_coordinates(self) -> np.ndarray:
        out = np.zeros((self.K, self.Np, 3))
        check(lib.dg_node_coordinates(self._h, _dptr(out)), "dg_node_coordinates")
        return out

    def set_coefficients(self, coef):
        p = _require_torch_device_tensor(coef, (self.K, self.ncoef), "coef")
        check(lib.dg_set_coefficients(self._h, p), "dg_set_coefficients")
        self.coef_generation = getattr(self, "coef_generation", 0) + 1
        self.last_coefficients = coef.detach().clone()

    def set_boundary(self, absorbing):
        """Absorbing unpaired faces: ``absorbing`` is a bool [K, 4] mask (True
        = absorbing; False = reflecting wall; faces with a neighbour must be
        False)."""
        kind = np.ascontiguousarray(np.asarray(absorbing, dtype=bool).astype(np.int32))
        if kind.shape != (self.K, 4):
            raise ValueError(f"absorbing mask has shape {kind.shape}, expected ({self.K}, 4)")
        check(lib.dg_set_boundary(self._h, _i32ptr(kind)), "dg_set_boundary")

    def set_fields(self, q):
        check(lib.dg_set_fields(self._h, _require_torch_device_tensor(q, self.field_shape, "q")), "dg_set_fields")

    def get_fields(self, out=None):
        out = self.empty_fields() if out is None else out
        check(lib.dg_get_fields(self._h, _require_torch_device_tensor(out, self.field_shape, "out")), "dg_get_fields")
        return out

    def set_state(self, q, r1, r2, step_index: int):
        z = C.c_void_p(0)
        p1 = _require_torch_device_tensor(r1, self.field_shape, "r1") if r1 is not None else z
        p2 = _require_torch_device_tensor(r2, self.field_shape, "r2") if r2 is not None else z
        check(
            lib.dg_set_state(self._h, _require_torch_device_tensor(q, self.field_shape, "q"), p1, p2, int(step_index)),
            "dg_set_state",
        )

    def get_state(self):
        q, r1, r2 = self.empty_fields(), self.empty_fields(), self.empty_fields()
        m = C.c_int64()
        check(
            lib.dg_get_state(
                self._h,
                C.c_void_p(q.data_ptr()), C.c_void_p(r1.data_ptr()), C.c_void_p(r2.data_ptr()), C.byref(m),
            ),
            "dg_get_state",
        )
        return q, (r1 if m.value >= 1 else None), (r2 if m.value >= 2 else None), m.value

    VARIANTS = {
        "valu": nat.DG_VARIANT_VALU,
        "mfma": nat.DG_VARIANT_MFMA,
        "mfma_bf16": nat.DG_VARIANT_MFMA_BF16,
        "mfma_f16": nat.DG_VARIANT_MFMA_F16,
        "elem": nat.DG_VARIANT_ELEM,
        "mfma_wide": nat.DG_VARIANT_MFMA_WIDE,
    }

    @property
    def variant(self) -> str:
        v = C.c_int()
        check(lib.dg_get_variant(self._h, C.byref(v)), "dg_get_variant")
        return {b: a for a, b in self.VARIANTS.items()}[v.value]

    @variant.setter
    def variant(self, name: str):
        check(lib.dg_set_variant(self._h, self.VARIANTS[name]), "dg_set_variant")

    @property
    def step_index(self) -> int:
        m = C.c_int64()
        check(lib.dg_step_index(self._h, C.byref(m)), "dg_step_index")
        return m.value

    def step(self, nsteps: int, dt: float):
        check(lib.dg_step(self._h, int(nsteps), float(dt)), "dg_step")

    def set_rate_classes(self, k_fast: int):
        """Elements [0, k_fast) take two half steps per step (two-rate
        stepping; 0 = single rate).  Restarts the Adams-Bashforth start-up."""
        check(lib.dg_set_rate_classes(self._h, int(k_fast)), "dg_set_rate_classes")

    def step_multirate(self, nsteps: int, dt: float):
        """``nsteps`` macro steps of size dt (the fast class takes 2 nsteps
        steps of dt/2)."""
        check(lib.dg_step_multirate(self._h, int(nsteps), float(dt)), "dg_step_multirate")

    def autotune(self, steps: int, dt: float, candidates=None) -> dict:
        """Times the built variants (all, or the names in ``candidates``) on
        this mesh and keeps the fastest.

        Returns microseconds per step by variant name (None where not built
        or not a candidate).  The timed steps write their fields into a
        scratch array, so the solver's state does not change.
        """
        import torch

        mask = 0
        if candidates is not None:
            for name in candidates:
                mask |= 1 << self.VARIANTS[name]
        us = np.zeros(nat.DG_NUM_VARIANTS)
        with torch.cuda.stream(self._stream):
            scratch = self.empty_fields()
        nbytes = scratch.numel() * scratch.element_size()
        check(
            lib.dg_autotune(self._h, int(steps), float(dt), mask, C.c_void_p(scratch.data_ptr()), nbytes, _dptr(us)),
            "dg_autotune",
        )
        names = {b: a for a, b in self.VARIANTS.items()}
        return {names[v]: (float(us[v]) if us[v] >= 0 else None) for v in range(nat.DG_NUM_VARIANTS)}

    def rhs(self, q, out=None):
        out = self.empty_fields() if out is None else out
        check(
            lib.dg_rhs(
                self._h,
                _require_torch_device_tensor(q, self.field_shape, "q"),
                _require_torch_device_tensor(out, self.field_shape, "out"),
            ),
            "dg_rhs",
        )
        return out

    def energy(self) -> float:
        e = C.c_double()
        check(lib.dg_energy(self._h, C.byref(e)), "dg_energy")
        return e.value

    def set_energy_tolerance(self, tol: float):
        """Growth tolerance of the energy stability check (negative: off)."""
        check(lib.dg_set_energy_tolerance(self._h, float(tol)), "dg_set_energy_tolerance")

    def debug_buffer(self, name: str) -> np.ndarray:
        """Copy of an internal device buffer (see dg_debug_buffer)."""
        nbytes = C.c_size_t(0)
        check(lib.dg_debug_buffer(self._h, name.encode(), None, C.byref(nbytes)), "dg_debug_buffer")
        dtype = np.int32 if name in ("conn", "fmask", "perm", "nodeface") else np.float32
        out = np.zeros(nbytes.value // 4, dtype=dtype)
        check(
            lib.dg_debug_buffer(self._h, name.encode(), out.ctypes.data_as(C.c_void_p), C.byref(nbytes)),
            "dg_debug_buffer",
        )
        return out

    def synchronize(self):
        check(lib.dg_synchronize(self._h), "dg_synchronize")

    def locate_points(self, xyz):
        """(element [n], Lagrange weights [n, Np]) of host points [n, 3]."""
        x = np.ascontiguousarray(np.atleast_2d(xyz), dtype=np.float64)
        elem = np.zeros(len(x), dtype=np.int64)
        w = np.zeros((len(x), self.Np))
        check(lib.dg_locate_points(self._h, len(x), _dptr(x), _i64ptr(elem), _dptr(w)), "dg_locate_points")
        return elem, w


class DGBatch:
    """Many solvers of one physics stepped together (one launch per degree
    and variant group and step; optionally replayed from a HIP graph).

    The batch keeps references to its members; they must stay open while it
    lives.
    """

    def __init__(self, members, stream=None, graph: bool = False):
        import torch

        self.members = list(members)
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        arr = (C.c_void_p * len(self.members))(*[m._h.value for m in self.members])
        members = C.cast(arr, C.POINTER(C.c_void_p))
        nbytes = C.c_size_t(0)
        check(lib.dg_batch_workspace_bytes(members, len(self.members), C.byref(nbytes)), "dg_batch_workspace_bytes")
        with torch.cuda.stream(stream):
            self._workspace = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        check(
            lib.dg_batch_create(
                members, len(self.members), C.c_void_p(self._workspace.data_ptr()), nbytes,
                C.c_void_p(stream.cuda_stream), C.byref(h),
            ),
            "dg_batch_create",
        )
        self._h = h
        if graph:
            self.set_graph(True)

    def close(self):
        if getattr(self, "_h", None):
            lib.dg_batch_destroy(self._h)
            self._h = None
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, enable: bool):
        check(lib.dg_batch_set_graph(self._h, int(bool(enable))), "dg_batch_set_graph")

    def step(self, nsteps: int, dt):
        dts = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (len(self.members),)))
        check(lib.dg_batch_step(self._h, int(nsteps), _dptr(dts)), "dg_batch_step")

    def groups(self):
        """[(degree, variant name, workgroups per launch)] of the launch groups."""
        n = C.c_int(0)
        check(lib.dg_batch_groups(self._h, C.byref(n), None, None, None), "dg_batch_groups")
        order = np.zeros(n.value, dtype=np.int32)
        variant = np.zeros(n.value, dtype=np.int32)
        tiles = np.zeros(n.value, dtype=np.int64)
        check(
            lib.dg_batch_groups(self._h, C.byref(n), _i32ptr(order), _i32ptr(variant), _i64ptr(tiles)),
            "dg_batch_groups",
        )
        names = {b: a for a, b in DGSolver.VARIANTS.items()}
        return [(int(o), names[int(v)], int(t)) for o, v, t in zip(order, variant, tiles)]
