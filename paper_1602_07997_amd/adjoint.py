"""Misfit of receiver traces and its coefficient gradient, as a torch
autograd function (marshalling only: the forward steps, the adjoint sweep
and the gradient accumulation run in the library's HIP kernels)."""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from ._native import check, lib
from .solver import DGSolver, _dptr, _require_torch_device_tensor


def ricker(t, f0: float, t0: float):
    """Ricker wavelet (1 - 2a) exp(-a), a = (pi f0 (t - t0))^2."""
    a = (np.pi * f0 * (np.asarray(t, dtype=float) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


class DGMisfit:
    """Point source + receivers + L2 misfit on a solver's mesh.

    ``wavelet`` holds f(t_m) for m = 0..nsteps; sources and receivers are
    host arrays of points [n, 3].  Traces and data are device float32
    [nsteps + 1, channels].
    """

    def __init__(self, solver: DGSolver, nsteps: int, dt: float, src_xyz, wavelet, rec_xyz,
                 checkpoint_every: int = 20):
        self.solver = solver
        self.nsteps, self.dt = int(nsteps), float(dt)
        src = np.ascontiguousarray(np.atleast_2d(src_xyz), dtype=np.float64) if src_xyz is not None else None
        rec = np.ascontiguousarray(np.atleast_2d(rec_xyz), dtype=np.float64)
        wav = np.ascontiguousarray(wavelet, dtype=np.float64) if src is not None else None
        if wav is not None and wav.shape != (self.nsteps + 1,):
            raise ValueError("wavelet must hold nsteps + 1 values")
        args = (
            solver._h, self.nsteps, self.dt, int(checkpoint_every),
            0 if src is None else len(src), None if src is None else _dptr(src),
            None if wav is None else _dptr(wav), len(rec), _dptr(rec),
        )
        nbytes = C.c_size_t(0)
        check(lib.dg_misfit_workspace_bytes(*args, C.byref(nbytes)), "dg_misfit_workspace_bytes")
        with torch.cuda.stream(solver._stream):
            self._workspace = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        check(
            lib.dg_misfit_create(*args, C.c_void_p(self._workspace.data_ptr()), nbytes, C.byref(h)),
            "dg_misfit_create",
        )
        self._h = h
        self.channels = int(lib.dg_misfit_channels(h))
        self._forwards = 0

    @property
    def generation(self):
        """Changes with every forward solve and every coefficient change of
        the solver: a gradient belongs to the forward of the same generation."""
        return (self._forwards, getattr(self.solver, "coef_generation", 0))

    def close(self):
        if getattr(self, "_h", None):
            lib.dg_misfit_destroy(self._h)
            self._h = None
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def trace_shape(self):
        return (self.nsteps + 1, self.channels)

    def forward(self, data=None):
        """(traces, J): receiver traces (device) and the misfit (0 without data)."""
        import torch

        traces = torch.empty(self.trace_shape, dtype=torch.float32, device="cuda")
        J = C.c_double(0.0)
        dp = _require_torch_device_tensor(data, self.trace_shape, "data") if data is not None else None
        check(
            lib.dg_misfit_forward(self._h, dp, _require_torch_device_tensor(traces, self.trace_shape, "traces"),
                                  C.byref(J)),
            "dg_misfit_forward",
        )
        self._forwards += 1
        return traces, J.value

    def gradient(self):
        """dJ/dcoef [K, ncoef] (device) for the last forward with data."""
        import torch

        s = self.solver
        g = torch.empty((s.K, s.ncoef), dtype=torch.float32, device="cuda")
        check(lib.dg_misfit_gradient(self._h, _require_torch_device_tensor(g, (s.K, s.ncoef), "grad")),
              "dg_misfit_gradient")
        return g


def _misfit_function():
    import torch

    class MisfitFunction(torch.autograd.Function):
        """J(coef): forward solve from the zero state with the given per-element
        coefficients; backward by the discrete adjoint."""

        @staticmethod
        def forward(ctx, coef, misfit, data):
            coef = coef.detach().contiguous().clone()
            misfit.solver.set_coefficients(coef)
            _, J = misfit.forward(data)
            ctx.misfit = misfit
            ctx.coef, ctx.data = coef, data
            ctx.generation = misfit.generation
            return torch.tensor(J, dtype=torch.float64, device=coef.device)

        @staticmethod
        def backward(ctx, gJ):
            f = ctx.misfit
            if f.generation != ctx.generation:
                # another forward solve or a coefficient change came between:
                # redo this call's forward solve so that the gradient belongs
                # to its coefficients and data, then restore the solver's
                # coefficients
                prev = getattr(f.solver, "last_coefficients", None)
                f.solver.set_coefficients(ctx.coef)
                f.forward(ctx.data)
                g = f.gradient()
                if prev is not None:
                    f.solver.set_coefficients(prev)
            else:
                g = f.gradient()
            return (g * gJ.to(g.dtype)), None, None

    return MisfitFunction


def misfit(coef, problem: DGMisfit, data):
    """Differentiable L2 misfit of the receiver traces against ``data``."""
    return _misfit_function().apply(coef, problem, data)
