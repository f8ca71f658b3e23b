"""ctypes binding of libdgwave.so (argument marshalling only).

Every function declared in ``include/dgwave.h`` is bound here under the same
name.  Importing this module raises ImportError when the library has not
been built: there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgwave.so")

DG_OK = 0
DG_E_ARG = -1
DG_E_SHAPE = -2
DG_E_MESH = -3
DG_E_STATE = -4
DG_E_HIP = -5
DG_E_UNSUPPORTED = -6
DG_E_UNSTABLE = -7
DG_ACOUSTIC = 0
DG_ELASTIC = 1
DG_ANISOTROPIC = 2
DG_VARIANT_VALU = 0
DG_VARIANT_MFMA = 1
DG_VARIANT_MFMA_BF16 = 2
DG_VARIANT_MFMA_F16 = 3
DG_VARIANT_ELEM = 4
DG_VARIANT_MFMA_WIDE = 5
DG_NUM_VARIANTS = 6
DG_BC_REFLECT = 0
DG_BC_ABSORB = 1

STATUS_NAMES = {
    DG_OK: "DG_OK",
    DG_E_ARG: "DG_E_ARG",
    DG_E_SHAPE: "DG_E_SHAPE",
    DG_E_MESH: "DG_E_MESH",
    DG_E_STATE: "DG_E_STATE",
    DG_E_HIP: "DG_E_HIP",
    DG_E_UNSUPPORTED: "DG_E_UNSUPPORTED",
    DG_E_UNSTABLE: "DG_E_UNSTABLE",
}

# torch ships its own HIP runtime (soname libamdhip64.so.7) and loads it by
# path.  Importing torch first makes the library's libamdhip64.so.7 dependency
# resolve to that same, already loaded runtime; loading the library first
# would bring in a second HIP/HSA runtime that cannot open the device.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1602_07997_amd.build_native`"
    )

lib = C.CDLL(LIB_PATH)

_p = C.c_void_p
_i64 = C.c_int64
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_szp = C.POINTER(C.c_size_t)

# name -> (restype, argtypes); mirrors include/dgwave.h
SIGNATURES = {
    "dg_abi_version": (C.c_int, []),
    "dg_last_error": (C.c_char_p, []),
    "dg_num_fields": (C.c_int, [C.c_int]),
    "dg_ref_sizes": (C.c_int, [C.c_int, _ip, _ip]),
    "dg_reference_operators": (C.c_int, [C.c_int, _dp, _dp, _dp, _dp, _i32p]),
    "dg_face_permutations": (C.c_int, [C.c_int, _i32p]),
    "dg_mesh_connectivity": (C.c_int, [_i64, _i64p, _i64p, _i32p, _i32p]),
    "dg_workspace_bytes": (C.c_int, [C.c_int, C.c_int, _i64, _szp]),
    "dg_create": (C.c_int, [C.c_int, C.c_int, _i64, _dp, _i64p, _p, C.c_size_t, _p, C.POINTER(_p)]),
    "dg_destroy": (None, [_p]),
    "dg_set_stream": (C.c_int, [_p, _p]),
    "dg_synchronize": (C.c_int, [_p]),
    "dg_set_variant": (C.c_int, [_p, C.c_int]),
    "dg_get_variant": (C.c_int, [_p, _ip]),
    "dg_node_coordinates": (C.c_int, [_p, _dp]),
    "dg_set_coefficients": (C.c_int, [_p, _p]),
    "dg_set_boundary": (C.c_int, [_p, _i32p]),
    "dg_set_fields": (C.c_int, [_p, _p]),
    "dg_get_fields": (C.c_int, [_p, _p]),
    "dg_set_state": (C.c_int, [_p, _p, _p, _p, _i64]),
    "dg_get_state": (C.c_int, [_p, _p, _p, _p, _i64p]),
    "dg_step_index": (C.c_int, [_p, _i64p]),
    "dg_step": (C.c_int, [_p, C.c_int, C.c_double]),
    "dg_set_rate_classes": (C.c_int, [_p, _i64]),
    "dg_step_multirate": (C.c_int, [_p, C.c_int, C.c_double]),
    "dg_rhs": (C.c_int, [_p, _p, _p]),
    "dg_energy": (C.c_int, [_p, _dp]),
    "dg_energy_noalloc": (C.c_int, [_p, _p]),
    "dg_set_energy_tolerance": (C.c_int, [_p, C.c_double]),
    "dg_debug_buffer": (C.c_int, [_p, C.c_char_p, _p, C.POINTER(C.c_size_t)]),
    "dg_autotune": (C.c_int, [_p, C.c_int, C.c_double, C.c_uint, _p, C.c_size_t, _dp]),
    "dg_batch_workspace_bytes": (C.c_int, [C.POINTER(_p), C.c_int, _szp]),
    "dg_batch_create": (C.c_int, [C.POINTER(_p), C.c_int, _p, C.c_size_t, _p, C.POINTER(_p)]),
    "dg_batch_destroy": (None, [_p]),
    "dg_batch_set_graph": (C.c_int, [_p, C.c_int]),
    "dg_batch_step": (C.c_int, [_p, C.c_int, _dp]),
    "dg_batch_groups": (C.c_int, [_p, _ip, _i32p, _i32p, _i64p]),
    "dg_locate_points": (C.c_int, [_p, _i64, _dp, _i64p, _dp]),
    "dg_misfit_workspace_bytes": (
        C.c_int, [_p, _i64, C.c_double, C.c_int, C.c_int, _dp, _dp, C.c_int, _dp, _szp]
    ),
    "dg_misfit_create": (
        C.c_int, [_p, _i64, C.c_double, C.c_int, C.c_int, _dp, _dp, C.c_int, _dp, _p, C.c_size_t, C.POINTER(_p)]
    ),
    "dg_misfit_destroy": (None, [_p]),
    "dg_misfit_channels": (_i64, [_p]),
    "dg_misfit_forward": (C.c_int, [_p, _p, _p, _dp]),
    "dg_misfit_gradient": (C.c_int, [_p, _p]),
}

for _name, (_res, _args) in SIGNATURES.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class DGError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.dg_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != DG_OK:
        raise DGError(status, where)
