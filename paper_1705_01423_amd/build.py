"""Build the HIP library libps_mi355x.so in-tree for gfx950 (hipcc, no JIT).

Each translation unit is compiled separately (in parallel), then linked into
one shared library next to this file.  Usage: ``python -m paper_1705_01423_amd.build``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.environ.get("PS_BUILD_DIR") or os.path.join(HERE, "_build")
LIB = os.environ.get("PS_LIB_OUT") or os.path.join(HERE, "libps_mi355x.so")
ARCH = os.environ.get("PS_OFFLOAD_ARCH", "gfx950")
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
# extra compile flags, e.g. launch-shape defines (-DPS_X_LDS=...) for tuning builds
EXTRA = os.environ.get("PS_EXTRA_FLAGS", "").split()

# (source, output object, extra defines)
UNITS = [
    ("api.hip", "api.o", []),
    ("fft_kernels.hip", "fft_f64.o", ["-DPS_FFT_T=double", "-DPS_FFT_PRIMARY=1"]),
    ("fft_kernels.hip", "fft_f32.o", ["-DPS_FFT_T=float"]),
    ("zsolve_kernels.hip", "zsolve.o", []),
    ("field_kernels.hip", "field.o", []),
    ("substep_kernels.hip", "substep.o", []),
    ("multires_kernels.hip", "multires.o", []),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return [
        "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
        # packed FP32 instructions stay disabled in all device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-I", os.path.join(HERE, "..", "include"),
    ] + EXTRA


def _compile(unit):
    src, obj, extra = unit
    srcp = os.path.join(CSRC, src)
    objp = os.path.join(BUILD, obj)
    cmd = [hipcc(), "-c", srcp, "-o", objp] + flags() + extra
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return objp


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = [u for u in UNITS if os.path.exists(os.path.join(CSRC, u[0]))]
    jobs = max(1, min(len(units), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    # ROCTx for the host-side trace ranges of the entry points
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC", "-L", ROCM_LIB,
                                                    "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
