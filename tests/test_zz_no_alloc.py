"""The allocation-free energy entry point against dg_energy, through the C ABI.

dg_energy_noalloc runs the energy kernels of dg_energy with their partial
sums in the library's static device array and writes the total to device
memory.  Same kernels, same workgroup split, same summation order: the two
must agree bit for bit.  Two calls in a row, the second on a smaller mesh,
check that the array's leftover contents from the first call do not leak
into the second; a mesh that needs more partial sums than the array holds is
refused before any device work.
"""

import ctypes as C

import numpy as np
import pytest
import torch

import dginputs as di
from paper_1602_07997_amd import _native as nat
from paper_1602_07997_amd.solver import DGSolver

pytestmark = pytest.mark.gpu


def _solver(physics, N, n, seed):
    mesh = di.kuhn_box(n, jitter=0.1, seed=seed)
    s = DGSolver(physics, N, mesh.elem_xyz, mesh.elem_topo)
    ncoef = 2 if physics == "acoustic" else 3
    rng = np.random.default_rng(seed)
    coef = np.exp(rng.uniform(np.log(0.5), np.log(2.0), size=(mesh.K, ncoef))).astype(np.float32)
    s.set_coefficients(torch.tensor(coef, device="cuda"))
    q = torch.tensor(rng.standard_normal((mesh.K, s.nfields, s.Np)).astype(np.float32), device="cuda")
    s.set_fields(q)
    return s


def _noalloc(s, out):
    return nat.lib.dg_energy_noalloc(s._h, C.c_void_p(out.data_ptr()))


def test_noalloc_energy_matches_dg_energy_two_calls():
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    big = _solver("elastic", 3, 6, seed=11)      # 1296 elements, 108 partial sums
    small = _solver("acoustic", 2, 2, seed=12)   # 48 elements, 2 partial sums
    for i, s in enumerate((big, small)):
        print(f"noalloc energy call {i}: {s.physics} N={s.order} K={s.K}", flush=True)
        nat.check(_noalloc(s, out[i:i + 1]), "dg_energy_noalloc")
        torch.cuda.synchronize()
        ref = s.energy()
        got = float(out[i].item())
        assert np.isfinite(got) and got > 0.0
        assert got == ref, (i, got, ref)
    # a step between two calls: the value follows the fields
    big.step(3, 1e-4)
    nat.check(_noalloc(big, out[0:1]), "dg_energy_noalloc")
    torch.cuda.synchronize()
    assert float(out[0].item()) == big.energy()
    big.close()
    small.close()


def test_noalloc_energy_refuses_oversized_mesh():
    # acoustic N = 5 takes 4 elements per energy workgroup: 73002 elements need
    # 18251 partial sums, above the 16384 of the static array
    mesh = di.kuhn_box(23, jitter=0.0, seed=0)
    s = DGSolver("acoustic", 5, mesh.elem_xyz, mesh.elem_topo)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = _noalloc(s, out)
    assert st == nat.DG_E_SHAPE
    assert b"16384" in nat.lib.dg_last_error()
    assert float(out.item()) == 0.0
    s.close()


def test_noalloc_energy_argument_errors():
    s = _solver("acoustic", 1, 2, seed=3)
    assert nat.lib.dg_energy_noalloc(s._h, None) == nat.DG_E_ARG
    assert nat.lib.dg_energy_noalloc(None, None) == nat.DG_E_ARG
    s.close()
