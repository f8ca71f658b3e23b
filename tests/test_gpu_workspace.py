"""Caller-owned device memory through the C ABI (GPU).

The library allocates no device memory: a solver, a batch and a misfit live
in torch uint8 workspaces sized by the *_workspace_bytes queries, and the
autotuner times its steps into a caller scratch array.  These tests check
the size checks, that a solver in a workspace of exactly the queried size
steps like the oracle, that coefficients are validated on the device, and
that the autotuner leaves the state bit for bit.
"""

import ctypes as C

import numpy as np
import pytest
import torch

import dginputs as di
from paper_1602_07997_amd import _native as nat
from paper_1602_07997_amd.solver import DGBatch, DGSolver, _dptr, _i64ptr
from tests._cases import Case

pytestmark = pytest.mark.gpu


def _bytes(physics, N, K):
    n = C.c_size_t(0)
    nat.check(nat.lib.dg_workspace_bytes(physics, N, K, C.byref(n)), "dg_workspace_bytes")
    return n.value


def _create_raw(mesh, N, ws, nbytes, physics=0):
    h = C.c_void_p()
    xyz = np.ascontiguousarray(mesh.elem_xyz)
    topo = np.ascontiguousarray(mesh.elem_topo)
    st = nat.lib.dg_create(
        physics, N, mesh.K, _dptr(xyz), _i64ptr(topo), C.c_void_p(ws.data_ptr()), nbytes,
        C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(h),
    )
    return st, h


def test_solver_in_exactly_sized_workspace_matches_oracle():
    c = Case("elastic", 3, 2, jitter=0.1, seed=21, coef_kind="random", init="gaussian")
    assert c.solver.workspace_bytes == _bytes(1, 3, c.mesh.K)
    c.check(c.to_host(c.solver.rhs(c.to_gpu(c.q0_gpu))), c.oracle.rhs(c.q0), 2e-6, "rhs")


def test_create_refuses_small_or_misaligned_workspace():
    mesh = di.kuhn_box(2, jitter=0.1, seed=1)
    need = _bytes(0, 2, mesh.K)
    ws = torch.zeros(need + 512, dtype=torch.uint8, device="cuda")
    st, h = _create_raw(mesh, 2, ws, need - 256)
    assert st == nat.DG_E_SHAPE and not h.value
    st, h = _create_raw(mesh, 2, ws[64:], need)
    assert st == nat.DG_E_ARG and not h.value
    # nothing was written into the refused buffer
    assert int(ws.count_nonzero()) == 0
    st, h = _create_raw(mesh, 2, ws, need)
    assert st == nat.DG_OK and h.value
    nat.lib.dg_destroy(h)


def test_two_solvers_in_one_buffer_do_not_overlap():
    """Workspaces are plain device memory: two solvers carved from the two
    halves of one torch buffer step independently and equal their twins."""
    mesh = di.kuhn_box(2, jitter=0.1, seed=2)
    need = _bytes(0, 3, mesh.K)
    buf = torch.empty(2 * need, dtype=torch.uint8, device="cuda")
    hs = []
    for half in (buf[:need], buf[need:]):
        st, h = _create_raw(mesh, 3, half, need)
        assert st == nat.DG_OK
        hs.append(h)
    twin = DGSolver("acoustic", 3, mesh.elem_xyz, mesh.elem_topo)
    coef = torch.tensor(di.acoustic_two_layer(mesh), dtype=torch.float32, device="cuda")
    q0 = torch.tensor(
        np.ascontiguousarray(np.moveaxis(di.acoustic_gaussian(twin.node_coordinates()), 0, 1), dtype=np.float32),
        device="cuda",
    )
    for i, h in enumerate(hs):
        nat.check(nat.lib.dg_set_coefficients(h, C.c_void_p(coef.data_ptr())), "coef")
        nat.check(nat.lib.dg_set_fields(h, C.c_void_p((q0 * (i + 1)).contiguous().data_ptr())), "fields")
        torch.cuda.synchronize()
    dt = di.time_step(mesh, 3, 1.5)
    for h in hs:
        nat.check(nat.lib.dg_step(h, 7, dt), "step")
    twin.set_coefficients(coef)
    twin.set_fields(q0)
    twin.step(7, dt)
    ref = twin.get_fields()
    for i, h in enumerate(hs):
        out = torch.empty_like(q0)
        nat.check(nat.lib.dg_get_fields(h, C.c_void_p(out.data_ptr())), "get")
        torch.cuda.synchronize()
        assert torch.equal(out, ref * (i + 1)) or torch.allclose(out, ref * (i + 1), rtol=1e-6, atol=1e-7)
    for h in hs:
        nat.lib.dg_destroy(h)
    twin.close()


def test_coefficients_validated_on_the_device():
    mesh = di.kuhn_box(2, jitter=0.1, seed=3)
    s = DGSolver("elastic", 2, mesh.elem_xyz, mesh.elem_topo)
    coef = torch.tensor(di.elastic_loguniform(mesh, 4), dtype=torch.float32, device="cuda")
    s.set_coefficients(coef)
    q = torch.zeros(s.field_shape, device="cuda")
    s.set_fields(q)
    s.step(1, 1e-3)
    for bad_value, where in ((-1.0, (17, 2)), (float("nan"), (40, 0)), (float("inf"), (5, 1)), (0.0, (0, 0))):
        bad = coef.clone()
        bad[where] = bad_value
        with pytest.raises(nat.DGError) as ei:
            s.set_coefficients(bad)
        assert ei.value.status == nat.DG_E_ARG
        assert f"coefficient {where[1]} of element {where[0]}" in str(ei.value)
        # a refused call leaves the solver without coefficients
        with pytest.raises(nat.DGError) as ei:
            s.step(1, 1e-3)
        assert ei.value.status == nat.DG_E_STATE
        s.set_coefficients(coef)
        s.step(1, 1e-3)
    # two bad entries: the first one is named
    bad = coef.clone()
    bad[30, 1] = -2.0
    bad[9, 2] = -3.0
    with pytest.raises(nat.DGError) as ei:
        s.set_coefficients(bad)
    assert "element 9" in str(ei.value)
    s.close()


def test_batch_refuses_small_workspace():
    mesh = di.kuhn_box(2, jitter=0.1, seed=5)
    members = [DGSolver("acoustic", N, mesh.elem_xyz, mesh.elem_topo) for N in (2, 3)]
    arr = (C.c_void_p * 2)(*[m._h.value for m in members])
    ptr = C.cast(arr, C.POINTER(C.c_void_p))
    n = C.c_size_t(0)
    nat.check(nat.lib.dg_batch_workspace_bytes(ptr, 2, C.byref(n)), "bytes")
    ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    st = nat.lib.dg_batch_create(ptr, 2, C.c_void_p(ws.data_ptr()), n.value - 256, None, C.byref(h))
    assert st == nat.DG_E_SHAPE and not h.value
    b = DGBatch(members)
    assert b._workspace.numel() == n.value
    b.close()
    for m in members:
        m.close()


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_autotune_leaves_the_state_untouched(physics):
    c = Case(physics, 4, 2, jitter=0.1, seed=6, coef_kind="random", init="gaussian")
    s = c.solver
    s.set_fields(c.to_gpu(c.q0_gpu))
    dt = c.dt
    s.step(3, dt)
    q, r1, r2, m = s.get_state()
    tr = s.debug_buffer("traces")
    us = s.autotune(2, dt)
    assert all(v is None or v > 0 for v in us.values())
    q2, r12, r22, m2 = s.get_state()
    assert m2 == m
    assert torch.equal(q, q2) and torch.equal(r1, r12) and torch.equal(r2, r22)
    assert np.array_equal(tr, s.debug_buffer("traces"))
