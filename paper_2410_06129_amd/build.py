"""Compile libpinv.so (HIP kernels + C-ABI) for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpinv.so")
SOURCES = ["pinv_gram.hip", "pinv_chol.hip", "pinv_trmm.hip", "pinv_apply.hip", "pinv_solve.hip",
           "pinv_metrics.hip", "pinv_api.hip", "pinv_serve.hip", "pinv_noalloc.hip", "pinv_eig.hip",
           "pinv_split.hip"]
SIM_LIB = os.path.join(HERE, "libpinv_schedsim.so")
HEADERS = ["pinv_device.h", "pinv_internal.h"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found; the HIP toolchain (ROCm) is required to build libpinv")


def build(verbose: bool = False) -> str:
    """Compile every source in parallel (always; no staleness shortcut) and link libpinv.so."""
    cc = hipcc()
    flags = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(HERE, "..", "include")]
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [cc, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
        objs.append(obj)
    errs = []
    for p, src in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            errs.append(f"--- {src} ---\n{text}")
        elif verbose and text.strip():
            print(text)
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    build_sim(verbose)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    return LIB


def build_sim(verbose: bool = False) -> str:
    """The serving scheduler on a simulated device (host C++ only, for CPU tests)."""
    cxx = shutil.which("g++") or "g++"
    tmp = SIM_LIB + ".tmp"
    cmd = [cxx, "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall",
           os.path.join(CSRC, "sched_sim.cpp"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("g++ failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, SIM_LIB)
    return SIM_LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
