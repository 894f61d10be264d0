"""Build libces.so (HIP for gfx950 + host C++) in-tree.

    python -m paper_1404_3773_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libces.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SOURCES = ["kernels.hip", "kernels_angular.hip", "kernels_radial.hip", "kernels_scf.hip",
           "kernels_mlp.hip", "kernels_block.hip", "kernels_kb.hip", "kernels_lobpcg.hip", "noalloc.hip", "capi.cpp", "lobpcg.cpp", "scf.cpp", "learned.cpp", "setup_tables.cpp"]

# Device code: gfx950 only; packed-FP32 instructions disabled.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          f"-I{os.path.join(ROOT, 'include')}", f"-I{ROCM}/include"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".", "_") + ".o")
        path = os.path.join(CSRC, src)
        if src.endswith(".hip"):
            cmd = [hipcc, "-x", "hip", *DEVICE_FLAGS, *COMMON, "-c", path, "-o", obj]
        else:
            cmd = [hipcc, *COMMON, "-D__HIP_PLATFORM_AMD__", "-c", path, "-o", obj]
        cmds.append(cmd)
        objs.append(obj)
    # one compiler process per source, at most 8 at once
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
        for f in [pool.submit(_run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", *DEVICE_FLAGS, "-o", tmp, *objs, f"-L{ROCM}/lib",
          "-lrocsolver", "-lrocblas", f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
