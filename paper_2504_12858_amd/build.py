"""Builds libgrainenv.so (HIP kernels + C ABI) for gfx950 with hipcc.

Flags: -ffp-contract=off keeps every floating-point expression as written
(explicit fmaf where a fused multiply-add is wanted), so the device position,
binning and distance functions give the same bits in every kernel; packed FP32
instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgrainenv.so")
# Host code under AddressSanitizer + UndefinedBehaviorSanitizer (CPU checks of
# the host-side paths only: parameter validation, sizes, saved-state checks).
LIB_SAN = os.path.join(HERE, "libgrainenv_san.so")
SOURCES = ["kernels.hip", "runtime.hip"]
ARCH = os.environ.get("GE_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    cmd = [hipcc(), "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-result",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    if sanitize:
        # Host code only: every sanitizer flag goes to the host pass.
        cmd += ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
                "-fno-omit-frame-pointer", "-shared-libsan"]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    cmd += ["-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
