"""Build libtimeevolve.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2205_15346_amd.build
"""

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtimeevolve.so")
SOURCES = ["arnoldi.hip", "stepper.hip", "sampling.hip", "api.hip", "engine.hip", "models.hip"]
ARCH = os.environ.get("TE_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found")
    return path


def build(verbose: bool = False) -> str:
    """Compile every HIP source into one shared library next to this file; returns its path."""
    out_tmp = LIB + ".tmp"
    cmd = [
        hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ] + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out_tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("hipcc failed building libtimeevolve.so")
    if verbose and proc.stderr:
        # the host pass does not know the packed-fp32 target feature; that warning is expected
        lines = [l for l in proc.stderr.splitlines() if "packed-fp32-ops" not in l]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
