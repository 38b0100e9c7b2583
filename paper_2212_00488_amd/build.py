"""Build of the HIP library (hipcc, gfx950) into the package directory."""

from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libstereo_mi355x.so")
SOURCES = [os.path.join(PKG, "csrc", n) for n in ("stereo.hip", "soft.hip", "server.hip", "calib.hip")]
HEADERS = [os.path.join(PKG, "csrc", n) for n in ("kernels.hip.h", "soft.hip.h", "context.h", "common.h",
                                                 "pipeline.h")] + [
    os.path.join(ROOT, "include", "stereo.h"), os.path.join(ROOT, "include", "stereo_calib.h")]


def hipcc_command(out: str = LIB) -> list[str]:
    return ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include"),
            # packed fp32 instructions stay off in all device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            *SOURCES, "-o", out]


def build() -> str:
    """Compile the library; always recompiles."""
    tmp = LIB + ".tmp"
    subprocess.check_call(hipcc_command(tmp))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
