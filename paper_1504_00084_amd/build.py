"""Build libmesh_sdd.so (HIP kernels for gfx950 + host runtime) in-tree.

    python -m paper_1504_00084_amd.build            # the library
    python -m paper_1504_00084_amd.build --probe    # and the VALU issue-cost probe

Packed-FP32 instructions are disabled for all device code
(``-Xclang -target-feature -Xclang -packed-fp32-ops``).
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmesh_sdd.so")
PROBE = os.path.join(PKG, "valu_probe")

ARCH = "gfx950"
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-result"]

SOURCES = [
    ("kernels.hip", ["--offload-arch=" + ARCH] + DEVICE_FLAGS),
    ("mesh_step.hip", ["--offload-arch=" + ARCH] + DEVICE_FLAGS),
    ("noalloc.hip", ["--offload-arch=" + ARCH] + DEVICE_FLAGS),
    ("runtime.cpp", []),
    ("mesh_step.cpp", []),
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
    cmd = [hipcc(), "-c"] + COMMON + extra + [os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), res.stdout, res.stderr))
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP / C++ source and link the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda a: _compile(*a), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), res.stdout, res.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_probe(verbose: bool = False) -> str:
    """Compile the stand-alone VALU issue-cost probe (the calibration of the
    roofline's slot weights; not part of the library)."""
    tmp = PROBE + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-O3", "-std=c++17", "--offload-arch=" + ARCH] + DEVICE_FLAGS + [
        os.path.join(CSRC, "valu_probe.hip"), "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("probe build failed: %s\n%s\n%s" % (" ".join(cmd), res.stdout, res.stderr))
    os.replace(tmp, PROBE)
    if verbose:
        print("built", PROBE)
    return PROBE


if __name__ == "__main__":
    build(verbose=True)
    if "--probe" in sys.argv[1:]:
        build_probe(verbose=True)
    sys.exit(0)
