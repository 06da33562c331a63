"""ctypes declarations of the C ABI in include/ps.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_size_t, c_uint, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PS_LIB_PATH") or os.path.join(HERE, "libps_mi355x.so")

PS_OK, PS_EINVAL, PS_ENOMEM, PS_EDEVICE, PS_ENOTCOMPAT, PS_ENONFINITE, PS_ENOTCONVERGED = range(7)
STATUS_NAMES = {0: "PS_OK", 1: "PS_EINVAL", 2: "PS_ENOMEM", 3: "PS_EDEVICE", 4: "PS_ENOTCOMPAT",
                5: "PS_ENONFINITE", 6: "PS_ENOTCONVERGED"}
PS_FP64, PS_FP32_REFINED, PS_FP32 = 0, 1, 2
PS_FLAG_STRICT_COMPAT, PS_FLAG_CHECK_FINITE = 1, 2
PS_CENTER, PS_FACE = 0, 1


class PsInfo(ctypes.Structure):
    _fields_ = [("iterations", c_int), ("rel_update", c_double), ("rel_residual", c_double),
                ("compat_defect", c_double), ("gauge_shift", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = c_void_p          # ps_plan_t
_D = c_void_p          # device pointer
_PP = POINTER(c_void_p)

SIGNATURES = {
    "poisson_plan_create": (c_int, [_PP, c_int, c_int, c_int, c_double, c_double, POINTER(c_double), c_int,
                                    c_double, c_int, c_uint]),
    "poisson_plan_workspace_bytes": (c_size_t, [_P]),
    "poisson_plan_set_workspace": (c_int, [_P, c_void_p, c_size_t]),
    "poisson_plan_destroy": (c_int, [_P]),
    "poisson_solve": (c_int, [_P, _D, _D, c_void_p, POINTER(PsInfo)]),
    "poisson_solve_static": (c_int, [_P, _D, _D, c_void_p, POINTER(PsInfo)]),
    "project": (c_int, [_P, _D, _D, _D, _D, _D, c_double, c_double, c_void_p, POINTER(PsInfo)]),
    "cn_solve": (c_int, [_P, c_int, c_double, _D, c_void_p]),
    "poisson_solve_adjoint": (c_int, [_P, _D, _D, c_void_p, POINTER(PsInfo)]),
    "project_adjoint": (c_int, [_P, _D, _D, _D, _D, _D, _D, _D, c_double, c_double, c_void_p, POINTER(PsInfo)]),
    "ps_cfl": (c_int, [_P, _D, _D, _D, _D, c_void_p]),
    "rk3_substep": (c_int, [_P, c_int, c_double, c_double, c_double, _D, _D, _D, _D, _D, _PP, _PP, c_void_p,
                            POINTER(PsInfo)]),
    "rk3_substep_adjoint": (c_int, [_P, c_int, c_double, c_double, c_double, _D, _D, _D, _D, _D, _PP, _PP, _PP,
                                    _PP, c_void_p, POINTER(PsInfo)]),
    "rk3_step_adjoint": (c_int, [_P, c_double, c_double, c_double, _D, _D, _D, _D, _D, _PP, _PP, c_void_p,
                                 POINTER(PsInfo)]),
    "rk3_step": (c_int, [_P, c_double, c_double, c_double, c_double, c_double, _D, _D, _D, _D, _D,
                         POINTER(c_double), c_void_p, POINTER(PsInfo)]),
    "ps_heat_flux": (c_int, [_P, _D, _D, c_double, _D, _D, c_void_p]),
    "mr_create": (c_int, [_PP, _P, c_int, c_int, c_int, c_int]),
    "mr_destroy": (c_int, [_P]),
    "mr_shape": (c_int, [_P, POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
    "mr_prolong_velocity": (c_int, [_P, _D, _D, _D, _D, _D, _D, c_void_p]),
    "mr_restrict_temperature": (c_int, [_P, _D, _D, c_void_p]),
    "mr_temperature_step": (c_int, [_P, c_double, c_double, _PP, _PP, _D, c_void_p]),
    "rk3_step_mr": (c_int, [_P, c_double, c_double, c_double, c_double, c_double, _D, _D, _D, _D, _D,
                            POINTER(c_double), c_void_p, POINTER(PsInfo)]),
    "ps_debug_stage": (c_int, [_P, c_int, _D, _D, c_void_p]),
    "ps_spectral_layout": (c_int, [_P, POINTER(c_int), POINTER(c_int)]),
    "ps_spectral_elems": (c_size_t, [_P]),
    "ps_stream_copy": (c_int, [_D, _D, c_size_t, c_void_p]),
    "ps_last_error": (ctypes.c_char_p, []),
}

_lib = None


class PsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libps_mi355x.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1705_01423_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != PS_OK:
        raise PsError(status, load().ps_last_error().decode())
    return status
