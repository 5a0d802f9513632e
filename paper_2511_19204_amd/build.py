"""Build libmppi.so (HIP for gfx950) in-tree with hipcc.

The kernels and the C-ABI host runtime are compiled together into one shared
library next to this file.  Packed-FP32 instruction selection is disabled
(-packed-fp32-ops) and fast-math is off; multiply-adds are contracted within one
expression only (-ffp-contract=on), so an inlined helper rounds the same way
in every kernel that uses it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("mppi_kernels.hip", "mppi_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", "mppi_dev.hpp"), os.path.join(ROOT, "include", "mppi.h")]
LIB = os.path.join(HERE, "libmppi.so")
ARCH = os.environ.get("MPPI_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fno-fast-math", "-ffp-contract=on", "-Wall", "-Wno-unused-function",
         "-I", os.path.join(ROOT, "include")]


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB):
        mt = os.path.getmtime(LIB)
        if all(os.path.getmtime(f) <= mt for f in SOURCES + HEADERS):
            return LIB
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, *SOURCES, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if noise not in ln and ln.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
