"""Build libannkin.so (HIP, gfx950) in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libannkin.so")

SOURCES = ["api.cpp", "jit.cpp", "jit_jac.cpp", "server.cpp", "source_kernels.hip",
           "deriv_kernels.hip", "integrate.hip", "kcnet.hip", "production.hip"]

# Packed FP32 instructions stay disabled: every float op is a plain VALU op.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-pthread",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(out: str = LIB, defines: dict | None = None, verbose: bool = False) -> str:
    """Compile every source into one shared library; returns its path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPFLAGS, "-shared", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for k, v in (defines or {}).items():
        cmd.append(f"-D{k}={v}")
    cmd += ["-o", tmp, *sources(), "-lhiprtc"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stderr[-4000:]}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
