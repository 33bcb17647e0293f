"""Build ``libubf.so`` (the C-ABI library) in-tree for gfx950.

Host C++ (plan builder, C ABI) is compiled with g++; the HIP kernels with
hipcc for gfx950 only; the shared object is linked with hipcc. Run as
``python -m paper_2501_04684_amd.build`` or call :func:`build`.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libubf.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HOST_SOURCES = ["plan.cpp", "capi.cpp", "solver.cpp"]
HIP_SOURCES = ["kernels.hip", "gmres.hip", "networks.hip", "noalloc.hip"]

HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-pthread", "-Wall", "-Wextra",
              "-Wno-unused-parameter", "-D__HIP_PLATFORM_AMD__",
              f"-I{ROCM}/include", f"-I{os.path.join(ROOT, 'include')}"]
# Packed FP32 VALU instructions are disabled for all device code.
HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=fast", f"-I{os.path.join(ROOT, 'include')}"]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


# Host-only sanitizer build (plan builder, C ABI, solver host code): the
# device code is the same objects as the product library.
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                  "-fno-sanitize-recover=undefined"]
SANITIZE_LIB = os.path.join(BUILD, "sanitize", "libubf.so")


def build(verbose: bool = True, sanitize: bool = False) -> str:
    """Compile every source and link ``libubf.so``; returns its path.

    ``sanitize=True`` builds the host C++ with AddressSanitizer and
    UndefinedBehaviorSanitizer into ``_build/sanitize/libubf.so`` instead
    (load it with ``UBF_LIBRARY`` set to that path and the sanitizer runtime
    preloaded); the HIP objects are the product's.
    """
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    out_dir = os.path.dirname(SANITIZE_LIB) if sanitize else BUILD
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        extra = SANITIZE_FLAGS if sanitize else []
        _run(["g++", *HOST_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        if not (sanitize and os.path.exists(obj)):
            _run([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    lib = SANITIZE_LIB if sanitize else LIB
    tmp = lib + ".tmp"
    link_extra = ["-lasan", "-lubsan"] if sanitize else []
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs,
          f"-L{ROCM}/lib", "-lamdhip64", "-lpthread", *link_extra])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
