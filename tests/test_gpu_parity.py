"""GPU hot path vs the FP64 oracle, through the C ABI (needs an MI355X).

Tolerances (float32 fields and operators against float64):
  * one right-hand-side evaluation: mass-weighted relative L2 <= 2e-6;
  * AB3 runs: relative L2 <= 1e-5 over all fields;
  * discrete energy: relative 1e-9 (float64 accumulation of the same
    float32-rounded input state).
"""

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.dg import AB3Stepper
from tests._cases import Case, log

pytestmark = pytest.mark.gpu

DEGREES = list(range(1, 9))


def _mesh_n(N):
    return 3 if N <= 4 else 2


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("N", DEGREES)
def test_rhs_parity(physics, N):
    log(f"rhs parity {physics} N={N}")
    c = Case(physics, N, _mesh_n(N), jitter=0.1, seed=N, coef_kind="random", init="smooth")
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    c.check(c.to_host(r), c.oracle.rhs(c.q0), 2e-6, "rhs")


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("N", DEGREES)
def test_steps_parity(physics, N):
    log(f"20-step parity {physics} N={N}")
    c = Case(physics, N, _mesh_n(N), jitter=0.1, seed=10 + N, coef_kind="random", init="gaussian")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(20, c.dt)
    q = c.to_host(c.solver.get_fields())
    c.check(q, AB3Stepper(c.oracle, c.q0).step(20, c.dt), 1e-5, "20 steps")


def test_config1_parity_100_steps():
    """Acoustic N=2 on the 8x8x8 Kuhn cube (3072 tets), rho = c = 1, walls,
    Gaussian pulse, 100 AB3 steps: FP32 GPU vs FP64 oracle."""
    log("config-1 parity (acoustic N=2, 3072 tets, 100 steps)")
    c = Case("acoustic", 2, 8, jitter=0.0, coef_kind="constant", init="gaussian")
    assert c.mesh.K == 3072
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(100, c.dt)
    q = c.to_host(c.solver.get_fields())
    st = AB3Stepper(c.oracle, c.q0)
    ref = st.step(100, c.dt)
    c.check(q, ref, 1e-5, "100 steps")
    e_gpu = c.solver.energy()
    e_ref = c.oracle.energy(ref)
    assert abs(e_gpu - e_ref) <= 1e-5 * e_ref


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("N", [1, 3, 8])
def test_energy_parity(physics, N):
    log(f"energy parity {physics} N={N}")
    c = Case(physics, N, _mesh_n(N), jitter=0.1, seed=30 + N, coef_kind="random", init="smooth")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    e = c.solver.energy()
    e_ref = c.oracle.energy(c.q0)
    assert abs(e - e_ref) <= 1e-9 * e_ref


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("N", [6, 7, 8])
def test_energy_parity_ragged_element_groups(physics, N):
    """30 elements: the energy kernel's element groups (8 or 4 elements per
    item from N = 6 / 7) and its tiles end part-way through."""
    log(f"energy parity, ragged groups, {physics} N={N}")
    c = Case(physics, N, 0, jitter=0.1, seed=40 + N, coef_kind="random", init="smooth", dims=(5, 1, 1))
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    e = c.solver.energy()
    e_ref = c.oracle.energy(c.q0)
    assert abs(e - e_ref) <= 1e-9 * e_ref


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_periodic_plane_wave_parity(physics):
    log(f"periodic parity {physics}")
    c = Case(physics, 3, 3, jitter=0.05, seed=3, coef_kind="random", periodic=True, init="smooth")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(30, c.dt)
    q = c.to_host(c.solver.get_fields())
    c.check(q, AB3Stepper(c.oracle, c.q0).step(30, c.dt), 1e-5, "30 periodic steps")


def test_ragged_tiles_and_tiny_meshes():
    """Meshes whose element count leaves a partial last tile, down to K=6."""
    for dims in [(1, 1, 1), (1, 1, 2), (2, 1, 3)]:
        for physics, N in (("acoustic", 2), ("elastic", 3), ("acoustic", 8)):
            log(f"ragged {dims} {physics} N={N}")
            c = Case(physics, N, 0, jitter=0.0, coef_kind="random", init="smooth", dims=dims)
            c.solver.set_fields(c.to_gpu(c.q0_gpu))
            c.solver.step(5, c.dt)
            q = c.to_host(c.solver.get_fields())
            c.check(q, AB3Stepper(c.oracle, c.q0).step(5, c.dt), 1e-5, "5 steps")


def test_determinism_and_resume():
    log("determinism / resume")
    c = Case("elastic", 4, 2, jitter=0.1, seed=5, coef_kind="random", init="gaussian")
    q0 = c.to_gpu(c.q0_gpu)
    c.solver.set_fields(q0)
    c.solver.step(40, c.dt)
    a = c.solver.get_fields().clone()
    c.solver.set_fields(q0)
    c.solver.step(40, c.dt)
    b = c.solver.get_fields().clone()
    assert torch.equal(a, b)
    # 15 steps, checkpoint, 25 more == 40 straight
    c.solver.set_fields(q0)
    c.solver.step(15, c.dt)
    q, r1, r2, m = c.solver.get_state()
    q, r1, r2 = q.clone(), r1.clone(), r2.clone()
    c.solver.set_fields(torch.zeros_like(q0))  # clobber
    c.solver.step(3, c.dt)
    c.solver.set_state(q, r1, r2, m)
    assert c.solver.step_index == 15
    c.solver.step(25, c.dt)
    d = c.solver.get_fields()
    assert torch.equal(a, d)


def test_energy_decays_and_nan_is_flagged():
    log("energy decay / non-finite detection")
    c = Case("acoustic", 3, 3, jitter=0.1, seed=8, coef_kind="layers", init="gaussian")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(1, c.dt)
    E = [c.solver.energy()]
    for _ in range(30):
        c.solver.step(1, c.dt)
        E.append(c.solver.energy())
    E = np.array(E)
    assert np.all(E[1:] <= E[:-1] * (1 + 1e-6))
    bad = c.to_gpu(c.q0_gpu)
    bad[3, 0, 2] = float("nan")
    c.solver.set_fields(bad)
    from paper_1602_07997_amd._native import DG_E_UNSTABLE, DGError

    with pytest.raises(DGError) as ei:
        c.solver.energy()
    assert ei.value.status == DG_E_UNSTABLE


def test_energy_growth_is_flagged_above_the_stable_step():
    """dt four times the step-size recipe (above the AB3 stability limit on
    this mesh; the FP64 oracle's energy grows by 4x per step within 30
    steps there): dg_energy flags the growth before the state overflows.
    At the recipe's dt the same checks pass for 30 steps."""
    from paper_1602_07997_amd._native import DG_E_UNSTABLE, DGError

    log("energy growth check")
    c = Case("acoustic", 3, 3, jitter=0.1, seed=8, coef_kind="layers", init="gaussian")
    for fac, expect in ((1.0, False), (4.0, True)):
        c.solver.set_fields(c.to_gpu(c.q0_gpu))
        c.solver.step(2, fac * c.dt)
        c.solver.energy()
        flagged = None
        for i in range(30):
            c.solver.step(1, fac * c.dt)
            try:
                e = c.solver.energy()
            except DGError as err:
                assert err.status == DG_E_UNSTABLE
                assert "grew" in str(err)
                flagged = i
                break
            assert np.isfinite(e)
        log(f"  dt x{fac}: flagged at step {flagged}")
        assert (flagged is not None) == expect
    # a disabled growth check only flags non-finite energies
    c.solver.set_energy_tolerance(-1.0)
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(12, 4.0 * c.dt)
    c.solver.energy()
    c.solver.step(1, 4.0 * c.dt)
    c.solver.energy()


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_device_tables_and_face_normals(physics):
    """Uploaded tables equal the host set-up, and the face normals the kernels
    form (seen through the v.n / s n traces) match the oracle's on all four
    faces; a compiler mis-selection once gave face 3 the face-1 normal."""
    import paper_1602_07997_amd as P
    from paper_1602_07997_amd.solver import mesh_connectivity

    N = 3
    log(f"device tables / normals {physics}")
    c = Case(physics, N, 3, jitter=0.1, seed=4, coef_kind="random", init="smooth")
    s, K = c.solver, c.mesh.K
    ops = P.reference_operators(N)
    e2e, e2f, orient = mesh_connectivity(c.mesh.elem_topo)
    conn = np.where(e2e < 0, (np.arange(K)[:, None] << 5) | 7, (e2e << 5) | (e2f.astype(np.int64) << 3) | orient)
    assert np.array_equal(s.debug_buffer("conn"), conn.astype(np.int32).ravel())
    assert np.array_equal(s.debug_buffer("perm"), ops["perm"].ravel())
    assert np.array_equal(s.debug_buffer("fmask"), ops["fmask"].ravel())
    np.testing.assert_allclose(s.debug_buffer("geo").reshape(K, 3, 3), c.geo.G, rtol=1e-6, atol=1e-6)
    nt = 2 if physics == "acoustic" else 6
    normals = np.zeros((K, 4, 3))
    for i in range(3):
        q = np.zeros_like(c.q0_gpu)
        if physics == "acoustic":
            q[:, 1 + i] = 1.0  # v = e_i: trace 1 is n_i
        else:
            q[:, 3 + i] = 1.0  # s_ii = 1 only: trace (3+i) is n_i
        s.rhs(c.to_gpu(q))
        torch.cuda.synchronize()
        tr = s.debug_buffer("traces_rhs").reshape(K, 4, nt, -1)
        normals[:, :, i] = tr[:, :, 1 if physics == "acoustic" else 3 + i, 0]
    for f in range(4):
        np.testing.assert_allclose(normals[:, f], c.geo.normals[:, f], atol=1e-6)


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("N", DEGREES)
def test_mfma_variant_parity(N, physics):
    """FP32 MFMA variant: one right-hand side and 20 AB3 steps against the
    oracle on 108 elements: at least three full tiles at every degree (tiles
    of 16, 32 or 64 elements) and a ragged last one."""
    log(f"mfma variant {physics} N={N}")
    c = Case(physics, N, 0, jitter=0.1, seed=50 + N, coef_kind="random", init="smooth", dims=(3, 2, 3))
    c.solver.variant = "mfma"
    assert c.solver.variant == "mfma"
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    c.check(c.to_host(r), c.oracle.rhs(c.q0), 2e-6, "rhs")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(20, c.dt)
    q = c.to_host(c.solver.get_fields())
    c.check(q, AB3Stepper(c.oracle, c.q0).step(20, c.dt), 1e-5, "20 steps")


@pytest.mark.parametrize("N", DEGREES)
def test_mfma_wide_tile_parity(N):
    """The other acoustic FP32 tile shape (twice the elements and wavefronts
    per workgroup from N = 4, half the elements below): one right-hand side
    and 20 AB3 steps on 160 elements (several full tiles of 32 or 64 and a
    ragged last one, or many small tiles), all six face orientations."""
    log(f"mfma wide tile acoustic N={N}")
    mesh = di.relabel_vertices(di.kuhn_box(3, 3, 2, jitter=0.1, seed=70 + N), seed=71 + N)
    c = Case("acoustic", N, 0, coef_kind="random", init="smooth", mesh=mesh, seed=70 + N)
    c.solver.variant = "mfma_wide"
    assert c.solver.variant == "mfma_wide"
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    c.check(c.to_host(r), c.oracle.rhs(c.q0), 2e-6, "rhs")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(20, c.dt)
    c.check(c.to_host(c.solver.get_fields()), AB3Stepper(c.oracle, c.q0).step(20, c.dt), 1e-5, "20 steps")


def test_mfma_wide_is_acoustic_only():
    from paper_1602_07997_amd._native import DG_E_UNSUPPORTED, DG_VARIANT_MFMA_WIDE, lib

    c = Case("elastic", 2, 1, jitter=0.0, coef_kind="random", init="smooth")
    assert lib.dg_set_variant(c.solver._h, DG_VARIANT_MFMA_WIDE) == DG_E_UNSUPPORTED


def test_unknown_variant_rejected():
    from paper_1602_07997_amd._native import DG_E_UNSUPPORTED, lib

    c = Case("elastic", 2, 1, jitter=0.0, coef_kind="random", init="smooth")
    assert lib.dg_set_variant(c.solver._h, 9) == DG_E_UNSUPPORTED
    assert lib.dg_set_variant(c.solver._h, -1) == DG_E_UNSUPPORTED
    assert c.solver.variant == "valu"


@pytest.mark.parametrize("physics,N", [("acoustic", 1), ("acoustic", 2), ("elastic", 1)])
def test_elem_variant_parity(physics, N):
    """Element-per-thread variant: one right-hand side and 20 AB3 steps
    against the oracle (ragged last block of 256 elements, walls)."""
    log(f"elem variant {physics} N={N}")
    c = Case(physics, N, 0, jitter=0.1, seed=60 + N, coef_kind="random", init="smooth", dims=(5, 4, 3))
    c.solver.variant = "elem"
    assert c.solver.variant == "elem"
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    c.check(c.to_host(r), c.oracle.rhs(c.q0), 2e-6, "rhs")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(20, c.dt)
    q = c.to_host(c.solver.get_fields())
    c.check(q, AB3Stepper(c.oracle, c.q0).step(20, c.dt), 1e-5, "20 steps")


def test_elem_variant_periodic_and_rejected_above_its_degrees():
    from paper_1602_07997_amd._native import DG_E_UNSUPPORTED, DGError

    c = Case("acoustic", 1, 3, jitter=0.0, coef_kind="random", init="smooth", periodic=True)
    c.solver.variant = "elem"
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(15, c.dt)
    c.check(c.to_host(c.solver.get_fields()), AB3Stepper(c.oracle, c.q0).step(15, c.dt), 1e-5, "15 steps")
    d = Case("elastic", 2, 1, jitter=0.0, coef_kind="random", init="smooth")
    with pytest.raises(DGError) as ei:
        d.solver.variant = "elem"
    assert ei.value.status == DG_E_UNSUPPORTED


@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
@pytest.mark.parametrize("variant,N,periodic", [
    ("elem", 1, False), ("valu", 2, False), ("valu", 4, True), ("valu", 6, False),
    ("mfma", 3, True), ("mfma", 5, False), ("mfma", 6, False), ("mfma", 8, False), ("mfma_f16", 4, False),
    ("mfma_bf16", 6, False),
])
def test_all_face_orientations_parity(physics, variant, N, periodic):
    """Elements whose vertices are listed in random even orders, so that
    shared faces meet under all six relative orientations (a Kuhn split alone
    gives two): one right-hand side and 20 AB3 steps against the oracle."""
    from dginputs import kuhn_box, relabel_vertices

    log(f"all orientations {physics} {variant} N={N} periodic={periodic}")
    mesh = relabel_vertices(kuhn_box(3, 2, 3, jitter=0.1, seed=80 + N, periodic=periodic), seed=90 + N)
    c = Case(physics, N, 0, coef_kind="random", init="smooth", mesh=mesh, seed=80 + N)
    c.solver.variant = variant
    assert c.solver.variant == variant
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    tol_r, tol_q = (1e-4, 1e-4) if variant in ("mfma_f16", "mfma_bf16") else (2e-6, 1e-5)
    c.check(c.to_host(r), c.oracle.rhs(c.q0), tol_r, "rhs")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(20, c.dt)
    q = c.to_host(c.solver.get_fields())
    c.check(q, AB3Stepper(c.oracle, c.q0).step(20, c.dt), tol_q, "20 steps")


@pytest.mark.parametrize("physics,N,dims,remap,split", [
    ("elastic", 7, (9, 9, 9), "0", "1"), ("elastic", 7, (9, 9, 9), "0", "0"), ("elastic", 8, (9, 9, 9), "1", "1"),
    ("elastic", 8, (9, 9, 9), "0", "1"), ("anisotropic", 7, (9, 9, 9), "1", "1"),
    ("anisotropic", 8, (9, 9, 9), "0", "1"),
    ("acoustic", 7, (11, 12, 12), "0", "1"), ("acoustic", 7, (11, 12, 12), "1", "1"),
    # ragged last tile inside a split last round: 258 tiles (the last with 4
    # elements) on 256 slots, and 515 tiles (the last with 8) on 512
    ("elastic", 8, (7, 7, 14), "0", "1"), ("acoustic", 7, (7, 7, 28), "0", "1"),
])
def test_mfma_short_last_round_parity(physics, N, dims, remap, split, monkeypatch):
    """Meshes whose 16-element tiles fill the MI355X's resident workgroups
    (256 compute units times one, or two for acoustic N = 7) once or twice
    plus a short last round (274 tiles for 256 slots, 594 for 512), with the
    tiles in launch order or (DGWAVE_XCD_REMAP=1, read when the solver is
    created) each XCD given a contiguous range of tiles, and the elastic
    kernels' last-round tiles split over two or three workgroups (launch
    order; DGWAVE_TAIL_SPLIT=0 keeps them whole): one RHS and 10 AB3 steps
    against the oracle."""
    log(f"short last round {physics} N={N} dims={dims} remap={remap} split={split}")
    monkeypatch.setenv("DGWAVE_XCD_REMAP", remap)
    monkeypatch.setenv("DGWAVE_TAIL_SPLIT", split)
    c = Case(physics, N, None, jitter=0.1, seed=95 + N, coef_kind="random", init="smooth", dims=dims)
    c.solver.variant = "mfma"
    r = c.solver.rhs(c.to_gpu(c.q0_gpu))
    torch.cuda.synchronize()
    c.check(c.to_host(r), c.oracle.rhs(c.q0), 2e-6, "rhs")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(10, c.dt)
    c.check(c.to_host(c.solver.get_fields()), AB3Stepper(c.oracle, c.q0).step(10, c.dt), 1e-5, "10 steps")


@pytest.mark.parametrize("physics,N,variant,dims", [
    ("elastic", 6, "mfma", (4, 4, 4)), ("elastic", 7, "mfma", (4, 4, 4)), ("elastic", 8, "mfma", (3, 4, 4)),
    ("elastic", 8, "mfma_f16", (3, 4, 4)), ("anisotropic", 8, "mfma", (3, 3, 4)),
    ("acoustic", 8, "mfma", (3, 4, 4)), ("acoustic", 8, "mfma_f16", (3, 4, 4)),
    ("acoustic", 7, "mfma", (3, 4, 4)), ("acoustic", 6, "mfma_wide", (4, 4, 4)),
])
def test_tail_split_matches_whole_tiles(physics, N, variant, dims, monkeypatch):
    """A mesh smaller than one round of workgroups: every tile of the MFMA
    kernels with more than four pairs (elastic N = 6..8, acoustic N = 6..8)
    shared by two or three workgroups, each taking a range of
    the tile's (node block, element block) pairs (default), or kept whole
    (DGWAVE_TAIL_SPLIT=0).  Each pair's arithmetic is the same either way, so
    the fields after 10 AB3 steps are identical; both against the oracle."""
    log(f"tail split {physics} N={N} {variant} dims={dims}")
    out = []
    for split in ("1", "0"):
        monkeypatch.setenv("DGWAVE_TAIL_SPLIT", split)
        c = Case(physics, N, None, jitter=0.1, seed=97 + N, coef_kind="random", init="smooth", dims=dims)
        c.solver.variant = variant
        c.solver.set_fields(c.to_gpu(c.q0_gpu))
        c.solver.step(10, c.dt)
        out.append(c.solver.get_fields().clone())
    assert torch.equal(out[0], out[1])
    tol = 1e-5 if variant == "mfma" else 1e-4
    c.check(c.to_host(out[0]), AB3Stepper(c.oracle, c.q0).step(10, c.dt), tol, "10 steps")
