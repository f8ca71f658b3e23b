"""Batched stepping of many meshes and the variant autotuner (needs an MI355X).

A batch member must follow exactly the trajectory it would follow alone:
each member is compared with a twin solver built from the same inputs and
stepped by itself with dg_step (relative L2 <= 1e-6; the kernels are the
same code, so in practice the results are identical), and every member is
also compared with the FP64 oracle at the AB3 tolerance (1e-5, or 1e-4 for
the split 16-bit variants).
"""

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.dg import AB3Stepper
from tests._cases import Case, log

pytestmark = pytest.mark.gpu

SAME = 1e-6


def _twin(c: Case, variant: str):
    from paper_1602_07997_amd import DGSolver

    t = DGSolver(c.physics, c.N, c.mesh.elem_xyz, c.mesh.elem_topo)
    t.set_coefficients(torch.tensor(c.coef, dtype=torch.float32, device="cuda"))
    t.variant = variant
    t.set_fields(c.to_gpu(c.q0_gpu))
    return t


def _members(physics, specs):
    """specs: [(N, dims, variant)] -> list of (Case, twin)."""
    out = []
    for i, (N, dims, variant) in enumerate(specs):
        c = Case(physics, N, None, jitter=0.1, seed=40 + i, coef_kind="random", init="gaussian", dims=dims)
        c.solver.variant = variant
        c.solver.set_fields(c.to_gpu(c.q0_gpu))
        out.append((c, _twin(c, variant)))
    return out


def _rel(a: torch.Tensor, b: torch.Tensor) -> float:
    a = a.double()
    b = b.double()
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


ACOUSTIC_SPECS = [(1, (3, 2, 2), "valu"), (2, (2, 3, 2), "valu"), (3, (3, 3, 2), "mfma"),
                  (3, (2, 2, 2), "valu"), (5, (2, 2, 3), "mfma"), (2, (4, 3, 3), "mfma"),
                  (4, (3, 2, 3), "mfma_wide"), (2, (3, 3, 2), "mfma_wide")]
ELASTIC_SPECS = [(1, (3, 2, 2), "valu"), (2, (2, 3, 2), "valu"), (4, (2, 2, 2), "valu"),
                 (2, (3, 3, 2), "valu"), (6, (3, 2, 3), "mfma"), (1, (3, 3, 2), "elem")]


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("physics", ["acoustic", "elastic"])
def test_batch_matches_individual(physics, graph):
    from paper_1602_07997_amd import DGBatch

    log(f"batch vs individual {physics} graph={graph}")
    pairs = _members(physics, ACOUSTIC_SPECS if physics == "acoustic" else ELASTIC_SPECS)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    batch = DGBatch([c.solver for c, _ in pairs], stream=stream, graph=graph)
    groups = batch.groups()
    log(f"  groups {groups}")
    assert sum(1 for _ in groups) == len({(c.N, c.solver.variant) for c, _ in pairs})
    dts = [c.dt for c, _ in pairs]
    nsteps = 20
    batch.step(nsteps, dts)
    for c, t in pairs:
        t.step(nsteps, c.dt)
    stream.synchronize()
    torch.cuda.synchronize()
    for c, t in pairs:
        assert c.solver.step_index == nsteps
        e = _rel(c.solver.get_fields(), t.get_fields())
        log(f"  N={c.N} {c.solver.variant} K={c.mesh.K}: batch vs alone {e:.2e}")
        assert e <= SAME
    for c, _ in pairs:
        ref = AB3Stepper(c.oracle, c.q0).step(nsteps, c.dt)
        c.check(c.to_host(c.solver.get_fields()), ref, 1e-5, f"member N={c.N} K={c.mesh.K} vs oracle")
    batch.close()


def test_batch_graph_replays_with_eager_work_between():
    """Replays of the captured six-step graph, with eager energy evaluations
    and host synchronisations between them, each checked against the eager
    twins."""
    from paper_1602_07997_amd import DGBatch

    log("batch graph replays")
    pairs = _members("acoustic", ACOUSTIC_SPECS[:4])
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    batch = DGBatch([c.solver for c, _ in pairs], stream=stream, graph=True)
    dts = [c.dt for c, _ in pairs]
    batch.step(2, dts)  # start-up steps, launched member by member
    for c, t in pairs:
        t.step(2, c.dt)
    for rep in range(4):
        batch.step(6, dts)
        for c, t in pairs:
            t.step(6, c.dt)
        stream.synchronize()
        torch.cuda.synchronize()
        for c, t in pairs:
            e = _rel(c.solver.get_fields(), t.get_fields())
            eb, et = c.solver.energy(), t.energy()
            assert e <= SAME, (rep, c.N, e)
            assert abs(eb - et) <= 1e-6 * abs(et)
        log(f"  replay {rep} ok")
    batch.close()


def test_batch_uneven_start_dt_change_and_variant_switch():
    """Members entering at different step indices, a change of dt, and a
    member switching kernel variant between batched calls."""
    from paper_1602_07997_amd import DGBatch

    log("batch uneven start / dt change / variant switch")
    pairs = _members("acoustic", ACOUSTIC_SPECS[:5])
    # member 1 is already 3 steps ahead, member 3 one step
    for idx, k in ((1, 3), (3, 1)):
        c, t = pairs[idx]
        c.solver.step(k, c.dt)
        t.step(k, c.dt)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    batch = DGBatch([c.solver for c, _ in pairs], stream=stream)
    dts = [c.dt for c, _ in pairs]
    batch.step(7, dts)
    for c, t in pairs:
        t.step(7, c.dt)
    dts2 = [0.9 * d for d in dts]
    batch.step(5, dts2)
    for (c, t), d in zip(pairs, dts2):
        t.step(5, d)
    stream.synchronize()
    torch.cuda.synchronize()
    c, t = pairs[2]
    c.solver.variant = "valu"
    t.variant = "valu"
    batch.step(4, dts2)
    for (c, t), d in zip(pairs, dts2):
        t.step(4, d)
    stream.synchronize()
    torch.cuda.synchronize()
    for c, t in pairs:
        assert c.solver.step_index == t.step_index
        e = _rel(c.solver.get_fields(), t.get_fields())
        log(f"  N={c.N} m={c.solver.step_index}: {e:.2e}")
        assert e <= SAME
    batch.close()


def test_batch_rejects_bad_members():
    from paper_1602_07997_amd import DGBatch
    from paper_1602_07997_amd._native import DGError

    a = Case("acoustic", 2, 2, seed=1)
    e = Case("elastic", 2, 2, seed=2)
    with pytest.raises(DGError):
        DGBatch([a.solver, e.solver])
    with pytest.raises(DGError):
        DGBatch([a.solver, a.solver])
    b = DGBatch([a.solver])
    with pytest.raises(DGError):  # no fields yet
        b.step(1, [a.dt])
    with pytest.raises(DGError):  # graphs need a non-default stream
        DGBatch([a.solver], stream=torch.cuda.default_stream(), graph=True)
    b.close()


@pytest.mark.parametrize("physics,N", [("acoustic", 3), ("acoustic", 6), ("elastic", 2)])
def test_autotune_keeps_state_and_picks_a_built_variant(physics, N):
    log(f"autotune {physics} N={N}")
    c = Case(physics, N, 3, jitter=0.1, seed=7, coef_kind="random", init="gaussian")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    c.solver.step(4, c.dt)
    q, r1, r2, m = c.solver.get_state()
    times = c.solver.autotune(3, c.dt)
    log(f"  us/step {times} -> {c.solver.variant}")
    assert times["valu"] is not None and times["valu"] > 0
    assert all(times[v] is not None for v in ("mfma", "mfma_bf16", "mfma_f16"))
    assert times[c.solver.variant] == min(v for v in times.values() if v is not None)
    q2, r12, r22, m2 = c.solver.get_state()
    torch.cuda.synchronize()
    assert m2 == m
    assert torch.equal(q, q2) and torch.equal(r1, r12) and torch.equal(r2, r22)
    # the traces were restored too: continuing gives the oracle's trajectory
    c.solver.step(6, c.dt)
    ref = AB3Stepper(c.oracle, c.q0).step(10, c.dt)
    tol = 1e-4 if c.solver.variant in ("mfma_bf16", "mfma_f16") else 1e-5
    c.check(c.to_host(c.solver.get_fields()), ref, tol, "after tuning, 10 steps")


def test_batch_recipe_shapes():
    """The batched workload's recipe at a reduced count: sizes are Kuhn boxes
    in range, degrees in {2..6}; a small batch built from it steps every
    member to the oracle's trajectory."""
    from paper_1602_07997_amd import DGBatch

    recipe = di.batch_recipe(count=6, seed=2, k_lo=200, k_hi=2000, n_lo=2, n_hi=4)
    for r in recipe:
        assert r["K"] == 6 * r["n"] ** 3 and 2 <= r["n"] <= 4 and 2 <= r["N"] <= 6
    cases = []
    for r in recipe:
        c = Case("acoustic", r["N"], r["n"], jitter=0.1, seed=r["mesh_seed"], coef_kind="random")
        c.solver.set_fields(c.to_gpu(c.q0_gpu))
        cases.append(c)
    for c in cases:
        c.solver.autotune(2, c.dt)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    batch = DGBatch([c.solver for c in cases], stream=stream, graph=True)
    batch.step(14, [c.dt for c in cases])
    stream.synchronize()
    torch.cuda.synchronize()
    for c in cases:
        ref = AB3Stepper(c.oracle, c.q0).step(14, c.dt)
        tol = 1e-4 if c.solver.variant in ("mfma_bf16", "mfma_f16") else 1e-5
        c.check(c.to_host(c.solver.get_fields()), ref, tol, f"member N={c.N} K={c.mesh.K} {c.solver.variant}")
    batch.close()


def test_autotune_candidate_mask():
    c = Case("acoustic", 4, 2, jitter=0.1, seed=8, coef_kind="random", init="gaussian")
    c.solver.set_fields(c.to_gpu(c.q0_gpu))
    times = c.solver.autotune(2, c.dt, ["valu"])
    assert times["valu"] is not None and all(times[v] is None for v in ("mfma", "mfma_bf16", "mfma_f16"))
    assert c.solver.variant == "valu"
    times = c.solver.autotune(2, c.dt, ["mfma", "mfma_bf16"])
    assert times["valu"] is None and times["mfma_f16"] is None
    assert c.solver.variant in ("mfma", "mfma_bf16")
