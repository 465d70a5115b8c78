"""Build libctrace.so (host C++ + gfx950 HIP kernels) in the package folder.

    python -m paper_2010_08482_amd.build_lib

Compiles every time it is called.  Objects go to paper_2010_08482_amd/_build.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libctrace.so")
BUILD = os.path.join(PKG, "_build")
ARCH = "gfx950"

# Packed-FP32 instructions stay off in every device compile.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + "\n".join(errs))
    if verbose and errs:
        print("\n".join(errs))


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    objs = []
    for src, extra in (("ctrace_kernels.hip", ["-x", "hip"]), ("ctrace_group.hip", ["-x", "hip"]),
                       ("ctrace_hist.hip", ["-x", "hip"]), ("ctrace_rdm.hip", ["-x", "hip"]),
                       ("ctrace_probe.hip", ["-x", "hip"]),
                       ("ctrace_host.cpp", ["-x", "hip"]), ("ctrace_server.cpp", ["-x", "hip"]),
                       ("ctrace_mc.cpp", ["-x", "hip"])):
        obj = os.path.join(BUILD, src + ".o")
        _run([cc, *COMMON, *DEVICE_FLAGS, *extra, "-c", os.path.join(SRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run([cc, *COMMON, "-shared", *objs, "-o", tmp, "-lpthread"], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
