"""Build libpmx.so: every HIP kernel compiled for gfx950 plus the host orchestration."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpmx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HIP_SOURCES = ["la_kernels.hip", "assemble_kernels.hip", "apply_kernels.hip", "mlp_kernels.hip", "learn.cpp",
               "tune.cpp", "factor.cpp"]
HOST_SOURCES = ["plan.cpp"]


def build(verbose=False):
    bdir = os.path.join(CSRC, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    objs = []
    for f in HIP_SOURCES:
        o = os.path.join(bdir, os.path.splitext(f)[0] + ".o")
        cmd = [HIPCC] + HIP_FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, f), "-o", o]
        procs.append((f, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(o)
    for f in HOST_SOURCES:
        o = os.path.join(bdir, os.path.splitext(f)[0] + ".o")
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", os.path.join(CSRC, f), "-o", o]
        procs.append((f, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(o)
    failed = []
    for f, cmd, p in procs:
        out, err = p.communicate()
        lines = [l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed.append(f)
            sys.stderr.write(f"--- {f} failed:\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            sys.stderr.write(f"--- {f}:\n" + "\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(failed))
    tmp = OUT + ".tmp"
    # -z defs: an unresolved symbol of the library's own (a missing template instantiation)
    # fails the link instead of the first load
    subprocess.run([HIPCC] + HIP_FLAGS + ["-shared", "-Wl,-z,defs", "-o", tmp] + objs, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
