"""Build step of the native library: hipcc for gfx950, in-tree output.

`build()` always recompiles (it is the "does it build" check);
`ensure_built()` compiles only when the library is missing or older than its
sources.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmc_cl.so")
SOURCES = [os.path.join(CSRC, "mc_cl.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("mc_dev.hpp", "mc_coop.hpp", "mc_kernels.hpp", "mc_ms.hpp")] + [
    os.path.join(ROOT, "include", "mc_cl.h")]
ARCH = os.environ.get("MC_CL_ARCH", "gfx950")


def hipcc_command(out: str = LIB) -> list:
    return [
        "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # no packed FP32 instructions in any HIP code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        "-o", out, *SOURCES,
    ]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    res = subprocess.run(hipcc_command(tmp), capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stdout, res.stderr)
    os.replace(tmp, LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(d) for d in DEPS):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
