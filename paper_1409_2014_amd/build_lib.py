"""Build the solver's shared library (libphisolve.so) in-tree for gfx950.

    python -m paper_1409_2014_amd.build_lib

Host-only sources are compiled with g++, the kernels with hipcc, in parallel,
then linked with hipcc.  Every call rebuilds from scratch.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(PKG, "lib")
LIBNAME = "libphisolve.so"
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 arithmetic in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__"]


def _run(cmd):
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"build step failed ({proc.returncode}): {' '.join(cmd)}\n{proc.stdout}")
    return proc.stdout


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    gxx = shutil.which("g++") or "g++"
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    incs = [f"-I{INCLUDE}", f"-I{CSRC}", f"-I{ROCM}/include"]
    jobs = []
    for src, compiler in (("plan_host.cpp", "gxx"), ("phi_api.cpp", "gxx"), ("ds_api.cpp", "gxx"),
                          ("solver_kernels.hip", "hipcc"), ("shared_kernels.hip", "hipcc"), ("batch_kernels.hip", "hipcc"),
                          ("ds_kernels.hip", "hipcc"), ("periodic_kernels.hip", "hipcc"),
                          ("scratch.hip", "hipcc")):
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        path = os.path.join(CSRC, src)
        if compiler == "gxx":
            cmd = [gxx, *HOST_FLAGS, *incs, "-c", path, "-o", obj]
        else:
            cmd = [hipcc, *HIP_FLAGS, *incs, "-c", path, "-o", obj]
        jobs.append((cmd, obj))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        outs = list(ex.map(lambda j: _run(j[0]), jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    out = os.path.join(LIBDIR, LIBNAME)
    tmp = out + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *[o for _, o in jobs], "-o", tmp,
          f"-L{ROCM}/lib", "-lamdhip64"])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv)
    print(path)
