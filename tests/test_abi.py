"""C-ABI checks that run without a GPU.

* the shared library loads and exports every function declared in
  include/dgwave.h, and the binding declares each one;
* host-side set-up (reference operators, face permutations, connectivity)
  matches the oracle's independently built counterparts;
* argument and mesh validation that happens before any device work.
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

import dginputs as di
from oracle.mesh import build_mesh
from oracle.refelem import reference_element
from paper_1602_07997_amd import _native as nat
from paper_1602_07997_amd.solver import mesh_connectivity, reference_operators

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "dgwave.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    names = _declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(nat.lib, name), name
        assert name in nat.SIGNATURES, name
    assert set(nat.SIGNATURES) == set(names)
    assert nat.lib.dg_abi_version() == 2
    assert nat.lib.dg_num_fields(0) == 4 and nat.lib.dg_num_fields(1) == 9 and nat.lib.dg_num_fields(2) == 9
    assert nat.lib.dg_num_fields(7) == -1


@pytest.mark.parametrize("N", range(1, 9))
def test_reference_operators_match_oracle(N):
    ops = reference_operators(N)
    ref = reference_element(N)
    np.testing.assert_allclose(ops["nodes"], ref.r, atol=1e-13)
    np.testing.assert_allclose(ops["D"], ref.D, atol=1e-11)
    np.testing.assert_allclose(ops["mass"], ref.M, atol=1e-13)
    np.testing.assert_allclose(ops["lift"], ref.LIFT, atol=1e-11)
    assert np.array_equal(ops["fmask"], ref.Fmask)


@pytest.mark.parametrize("N", [1, 4, 8])
def test_product_operators_differentiate_monomials(N):
    ops = reference_operators(N)
    r, s, t = ops["nodes"].T
    for a in range(N + 1):
        for b in range(N + 1 - a):
            c = N - a - b
            u = r**a * s**b * t**c
            du = a * r ** max(a - 1, 0) * s**b * t**c
            np.testing.assert_allclose(ops["D"][0] @ u, du, atol=1e-11)


@pytest.mark.parametrize("relabel", [False, True])
@pytest.mark.parametrize("periodic", [False, True])
def test_connectivity_and_face_permutations_match_oracle(periodic, relabel):
    m = di.kuhn_box(3, 4, 3, jitter=0.1, seed=7, periodic=periodic)
    if relabel:  # random even vertex orders: shared faces meet in all six orientations
        m = di.relabel_vertices(m, seed=9)
    for N in (2, 5):
        geo = build_mesh(N, m.elem_xyz, m.elem_topo, m.period)
        e2e, e2f, orient = mesh_connectivity(m.elem_topo)
        assert np.array_equal(e2e, geo.EToE)
        assert np.array_equal(e2f, geo.EToF)
        perm = reference_operators(N)["perm"]
        k, f = np.nonzero(~geo.wall)
        assert np.all(orient[k, f] >= 0)
        assert np.array_equal(perm[orient[k, f]], geo.nbr_node[k, f])
        assert np.all(orient[geo.wall] == -1)
        assert set(np.unique(orient[k, f]).tolist()) == (set(range(6)) if relabel else {0, 1})


def test_mass_matrix_is_exactly_symmetric():
    # the energy kernel reads row n of M as column n
    for N in range(1, 9):
        M = reference_operators(N)["mass"]
        assert np.array_equal(M, M.T)


def test_permutations_are_permutations():
    for N in range(1, 9):
        perm = reference_operators(N)["perm"]
        Nfp = (N + 1) * (N + 2) // 2
        for o in range(6):
            assert sorted(perm[o]) == list(range(Nfp))
        assert np.array_equal(perm[0], np.arange(Nfp))


def test_host_validation_errors():
    bad = C.c_int()
    assert nat.lib.dg_ref_sizes(0, C.byref(bad), C.byref(bad)) == nat.DG_E_UNSUPPORTED
    assert nat.lib.dg_ref_sizes(9, C.byref(bad), C.byref(bad)) == nat.DG_E_UNSUPPORTED
    assert "order" in nat.lib.dg_last_error().decode()
    # a face shared by three elements
    topo = np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]], dtype=np.int64)
    with pytest.raises(nat.DGError) as ei:
        mesh_connectivity(topo)
    assert ei.value.status == nat.DG_E_MESH
    topo = np.array([[0, 1, 1, 3]], dtype=np.int64)
    with pytest.raises(nat.DGError):
        mesh_connectivity(topo)


# A stand-in workspace address: 256-byte aligned, never dereferenced, since
# every check below fails (or the size check refuses it) before device work.
FAKE_WS = C.c_void_p(1 << 20)


def _create(physics, order, xyz, topo, ws=FAKE_WS, ws_bytes=0):
    h = C.c_void_p()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    topo = np.ascontiguousarray(topo, dtype=np.int64)
    st = nat.lib.dg_create(
        physics, order, xyz.shape[0], xyz.ctypes.data_as(C.POINTER(C.c_double)),
        topo.ctypes.data_as(C.POINTER(C.c_int64)), ws, ws_bytes, None, C.byref(h),
    )
    return st, h


def _ws_bytes(physics, order, K):
    n = C.c_size_t(0)
    st = nat.lib.dg_workspace_bytes(physics, order, K, C.byref(n))
    return st, n.value


@pytest.mark.parametrize("physics", [0, 1, 2])
@pytest.mark.parametrize("N", [1, 4, 8])
def test_workspace_bytes_cover_every_array(physics, N):
    """The workspace holds q, the three-slot AB3 ring, three trace buffers and
    the per-element and operator tables, each 256-byte aligned."""
    Np, Nfp = (N + 1) * (N + 2) * (N + 3) // 6, (N + 1) * (N + 2) // 2
    NF, NT = (4, 2) if physics == 0 else (9, 6)
    for K in (1, 48, 1000):
        st, n = _ws_bytes(physics, N, K)
        assert st == nat.DG_OK
        assert n % 256 == 0
        floor = 4 * (4 * K * NF * Np + 3 * K * 4 * NT * Nfp + 9 * K) + 8 * K
        assert n >= floor
    # the operator tables do not grow with K; per element: q and three ring
    # slots, three trace buffers, G, derived and raw coefficients, four face
    # words, J and at most one energy partial sum
    CB, ncoef = {0: (8, 2), 1: (16, 3), 2: (32, 22)}[physics]
    per_elem = 4 * (4 * NF * Np + 3 * 4 * NT * Nfp + 9 + CB + ncoef + 4) + 8
    _, n1 = _ws_bytes(physics, N, 1000)
    _, n2 = _ws_bytes(physics, N, 2000)
    delta = (n2 - n1) - 1000 * per_elem
    assert -32 * 256 <= delta <= 1000 * 8 + 32 * 256  # alignment of each array, energy partial sums
    if physics == 2:  # the elastic tables, and more coefficient words per element
        assert _ws_bytes(2, N, 1000)[1] > _ws_bytes(1, N, 1000)[1]


def test_workspace_bytes_argument_errors():
    assert _ws_bytes(0, 2, 0)[0] == nat.DG_E_ARG
    assert _ws_bytes(0, 2, 1 << 26)[0] == nat.DG_E_ARG
    assert _ws_bytes(3, 2, 10)[0] == nat.DG_E_ARG
    assert _ws_bytes(0, 9, 10)[0] == nat.DG_E_UNSUPPORTED
    assert nat.lib.dg_workspace_bytes(0, 2, 10, None) == nat.DG_E_ARG


def test_create_checks_the_workspace_before_device_work():
    m = di.kuhn_box(2)
    _, need = _ws_bytes(0, 2, m.K)
    st, h = _create(0, 2, m.elem_xyz, m.elem_topo, ws=FAKE_WS, ws_bytes=need - 1)
    assert st == nat.DG_E_SHAPE and not h.value
    assert str(need) in nat.lib.dg_last_error().decode()
    st, h = _create(0, 2, m.elem_xyz, m.elem_topo, ws=C.c_void_p((1 << 20) + 64), ws_bytes=need)
    assert st == nat.DG_E_ARG and "aligned" in nat.lib.dg_last_error().decode()
    st, h = _create(0, 2, m.elem_xyz, m.elem_topo, ws=None, ws_bytes=need)
    assert st == nat.DG_E_ARG


def test_library_never_allocates_device_memory():
    """Device memory comes from the caller: no allocation call in the sources
    (the static array of the allocation-free energy entry point is not one)."""
    csrc = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1602_07997_amd", "csrc")
    pat = re.compile(r"\b(hipMalloc\w*|hipFree\w*|hipExtMalloc\w*|hipHostMalloc|hipMallocManaged)\s*\(")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".cpp", ".hip", ".hpp", ".h")):
            text = re.sub(r"//[^\n]*", "", open(os.path.join(csrc, name)).read())
            assert not pat.search(text), name


def test_create_rejects_bad_meshes_before_device_work():
    m = di.kuhn_box(2)
    st, h = _create(5, 2, m.elem_xyz, m.elem_topo)
    assert st == nat.DG_E_ARG and not h.value
    st, h = _create(0, 9, m.elem_xyz, m.elem_topo)
    assert st == nat.DG_E_UNSUPPORTED
    xyz = m.elem_xyz.copy()
    xyz[5, [2, 3]] = xyz[5, [3, 2]]  # invert one element
    st, h = _create(0, 2, xyz, m.elem_topo)
    assert st == nat.DG_E_MESH and "Jacobian" in nat.lib.dg_last_error().decode()
    # ids say the faces match but the coordinates do not
    xyz = m.elem_xyz.copy()
    topo = m.elem_topo.copy()
    xyz[0] += 0.01 * np.array([[0, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 1.0]])
    st, h = _create(0, 2, xyz, topo)
    assert st == nat.DG_E_MESH


def test_empty_and_oversized_meshes_rejected():
    """K = 0 and K >= 2^26 are rejected before any device work (the per-face
    connectivity word packs the neighbour index in 26 bits)."""
    empty_xyz = np.zeros((0, 4, 3))
    empty_topo = np.zeros((0, 4), dtype=np.int64)
    st, h = _create(0, 2, empty_xyz, empty_topo)
    assert st == nat.DG_E_ARG and not h.value
    e2e = np.zeros((1, 4), dtype=np.int64)
    e2f = np.zeros((1, 4), dtype=np.int32)
    assert nat.lib.dg_mesh_connectivity(
        0, empty_topo.ctypes.data_as(C.POINTER(C.c_int64)), e2e.ctypes.data_as(C.POINTER(C.c_int64)),
        e2f.ctypes.data_as(C.POINTER(C.c_int32)), e2f.ctypes.data_as(C.POINTER(C.c_int32)),
    ) == nat.DG_E_ARG
    one = di.kuhn_box(1)
    h = C.c_void_p()
    st = nat.lib.dg_create(
        0, 2, 1 << 26, one.elem_xyz.ctypes.data_as(C.POINTER(C.c_double)),
        one.elem_topo.ctypes.data_as(C.POINTER(C.c_int64)), FAKE_WS, 1 << 40, None, C.byref(h),
    )
    assert st == nat.DG_E_ARG and not h.value


def test_batch_and_misfit_entry_points_reject_null_arguments():
    out = C.c_void_p()
    nb = C.c_size_t(0)
    assert nat.lib.dg_batch_create(None, 0, FAKE_WS, 0, None, C.byref(out)) == nat.DG_E_ARG
    assert nat.lib.dg_batch_workspace_bytes(None, 0, C.byref(nb)) == nat.DG_E_ARG
    assert nat.lib.dg_batch_step(None, 1, None) == nat.DG_E_ARG
    assert nat.lib.dg_autotune(None, 1, 1.0, 0, None, 0, None) == nat.DG_E_ARG
    assert nat.lib.dg_misfit_create(None, 10, 0.1, 5, 0, None, None, 1, None, FAKE_WS, 0,
                                    C.byref(out)) == nat.DG_E_ARG
    assert nat.lib.dg_misfit_workspace_bytes(None, 10, 0.1, 5, 0, None, None, 1, None, C.byref(nb)) == nat.DG_E_ARG
    assert nat.lib.dg_misfit_forward(None, None, None, None) == nat.DG_E_ARG
    assert nat.lib.dg_misfit_gradient(None, None) == nat.DG_E_ARG
    assert nat.lib.dg_misfit_channels(None) == -1
    n = C.c_int(0)
    assert nat.lib.dg_batch_groups(None, C.byref(n), None, None, None) == nat.DG_E_ARG
    assert nat.lib.dg_locate_points(None, 1, None, None, None) == nat.DG_E_ARG
