"""Host-side checks of the C ABI: the library loads and exports every declared symbol,
and argument validation rejects bad input before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1705_01423_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ps.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:ps_status|size_t|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("poisson_plan_create", "poisson_solve", "project", "cn_solve", "poisson_solve_adjoint",
              "project_adjoint", "rk3_substep", "rk3_substep_adjoint", "rk3_step", "rk3_step_adjoint",
              "poisson_solve_static", "ps_heat_flux",
              "ps_debug_stage", "ps_last_error"):
        assert n in names


def test_library_exports_all_symbols():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) <= set(_lib.SIGNATURES)


def test_library_marks_trace_ranges():
    """Every entry point opens a ROCTx range (host-side trace annotation): the library
    imports the range calls from the ROCTx runtime."""
    import shutil
    import subprocess
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    out = subprocess.run(["nm", "-D", "--undefined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
    src = open(os.path.join(ROOT, "paper_1705_01423_amd", "csrc", "api.hip")).read()
    for n in ("poisson_solve", "project", "rk3_substep", "rk3_step", "rk3_step_adjoint", "rk3_step_mr"):
        assert f'PS_RANGE("{n}")' in src, n


def _create(nx, ny, nz, zf=None, prec=0):
    lib = _lib.load()
    zf = np.linspace(0, 1, nz + 1) if zf is None else zf
    zf = np.ascontiguousarray(zf, dtype=np.float64)
    h = ctypes.c_void_p()
    st = lib.poisson_plan_create(ctypes.byref(h), nx, ny, nz, 1.0, 1.0,
                                 zf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), prec, 0.0, 0, 0)
    return st, lib.ps_last_error().decode()


@pytest.mark.parametrize("dims,msg", [((5, 8, 8), "nx"), ((10, 8, 8), "nx"), ((8, 7, 8), "ny"),
                                      ((8, 8, 1), "nz"), ((8, 8, 4096), "nz"), ((8192, 8, 8), "nx"),
                                      ((18, 8, 8), "nx"), ((8, 9, 8), "ny"), ((20, 8, 8), "nx")])
def test_plan_rejects_bad_dims(dims, msg):
    st, err = _create(*dims)
    assert st == _lib.PS_EINVAL and msg in err


def test_plan_rejects_bad_grid():
    zf = np.linspace(0, 1, 9)
    zf[4] = zf[3]
    st, err = _create(8, 8, 8, zf)
    assert st == _lib.PS_EINVAL and "increasing" in err
    zf = np.linspace(0, 1, 9)
    zf[2] = np.nan
    st, err = _create(8, 8, 8, zf)
    assert st == _lib.PS_EINVAL and "finite" in err
    st, err = _create(8, 8, 8, prec=7)
    assert st == _lib.PS_EINVAL and "precision" in err


def test_null_plan_rejected():
    lib = _lib.load()
    st = lib.poisson_solve(None, ctypes.c_void_p(16), ctypes.c_void_p(32), None, None)
    assert st == _lib.PS_EINVAL
    assert lib.poisson_plan_destroy(None) == _lib.PS_OK


def test_null_plan_rejected_by_every_entry_point():
    """Every field entry point validates the plan before touching the device."""
    lib = _lib.load()
    d = ctypes.c_void_p(256)
    st = lib.rk3_step(None, 0.0, 1.3, 1.0, 1e-3, 1e-3, d, d, d, d, d, None, None, None)
    assert st == _lib.PS_EINVAL
    assert lib.ps_heat_flux(None, d, d, 1e-3, d, d, None) == _lib.PS_EINVAL
    assert lib.project(None, d, d, d, d, None, 1.0, 0.0, None, None) == _lib.PS_EINVAL
    assert lib.cn_solve(None, 0, 1e-3, d, None) == _lib.PS_EINVAL
    assert lib.ps_cfl(None, d, d, d, d, None) == _lib.PS_EINVAL
    assert "plan" in lib.ps_last_error().decode()
