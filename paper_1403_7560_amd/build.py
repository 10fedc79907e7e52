"""Build libswmc.so (HIP kernels + host runtime) for gfx950 with hipcc.

Run as `python -m paper_1403_7560_amd.build`; the library lands next to this
file so that it travels with the source tree.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libswmc.so")

ARCH = os.environ.get("SWMC_ARCH", "gfx950")
# -ffp-contract=off: the XY bond test and mirror are evaluated operation by
# operation, exactly as written.  Packed FP32 instructions are disabled.
DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"--offload-arch={ARCH}",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wno-unused-variable", "-Wno-unused-but-set-variable"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-variable"]


def hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libswmc")
    return h


def build(verbose=False):
    """Compile every kernel translation unit (in parallel) and the host
    runtime, then link them into libswmc.so."""
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    hips = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    objs, compiles = [], []
    for f in hips:
        o = os.path.join(BUILD, f[:-4] + ".o")
        objs.append(o)
        compiles.append([cc, "-c", os.path.join(CSRC, f), "-o", o] + DEVICE_FLAGS)
    eobj = os.path.join(BUILD, "sw_engine.o")
    objs.append(eobj)
    compiles.append([cc, "-c", os.path.join(CSRC, "sw_engine.cpp"), "-o", eobj] + HOST_FLAGS)
    procs = []
    for cmd in compiles:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = None
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed = failed or cmd
    if failed:
        raise RuntimeError(f"build step failed: {' '.join(failed[:3])}")
    link = [cc, "-shared", f"--offload-arch={ARCH}", "-fPIC"] + objs + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link step failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
