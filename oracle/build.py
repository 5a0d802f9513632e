"""Build the CPU oracle (test infrastructure only) into oracle/liboracle.so.

Plain g++ with OpenMP, no fast-math and no FMA contraction, so the FP64
reference rounds every operation as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mppi_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build(force: bool = True, sanitize: bool = False) -> str:
    """sanitize=True: the same source with AddressSanitizer and
    UndefinedBehaviorSanitizer (oracle/liboracle_san.so, host code only); load
    it with ORACLE_LIB and the sanitizer runtimes preloaded."""
    lib = LIB_SAN if sanitize else LIB
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(SRC):
        return lib
    tmp = lib + ".tmp"
    opt = ["-O1", *SANITIZE] if sanitize else ["-O2"]
    cmd = ["g++", *opt, "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def sanitizer_runtimes() -> list:
    """Paths of the compiler's ASan and UBSan runtimes (for LD_PRELOAD)."""
    out = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True, check=True).stdout.strip()
        out.append(p)
    return out


if __name__ == "__main__":
    import sys
    print(build(sanitize="--sanitize" in sys.argv))
