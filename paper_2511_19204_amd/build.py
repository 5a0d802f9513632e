"""Build libmppi.so (HIP for gfx950) in-tree with hipcc.

The kernels and the C-ABI host runtime are compiled together into one shared
library next to this file.  Packed-FP32 instruction selection is disabled
(-packed-fp32-ops) and fast-math is off; multiply-adds are contracted within one
expression only (-ffp-contract=on), so an inlined helper rounds the same way
in every kernel that uses it.

The compiler's per-kernel resource remarks are checked: no kernel may use
scratch memory (register spills), and the body-schedule rollout kernel and every
persistent kernel must fit two wavefronts per SIMD (at most 256 VGPRs), which
launches of more than one wavefront per SIMD rely on (the persistent forms size
their grids to the occupancy they get).
"""
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("mppi_kernels.hip", "mppi_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", "mppi_dev.hpp"), os.path.join(ROOT, "include", "mppi.h")]
LIB = os.path.join(HERE, "libmppi.so")
LIB_SAN = os.path.join(HERE, "libmppi_san.so")
ARCH = os.environ.get("MPPI_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fno-fast-math", "-ffp-contract=on", "-Wall", "-Wno-unused-function",
         "-I", os.path.join(ROOT, "include")]


def resource_usage(remarks: str) -> dict:
    """{kernel: {"VGPRs": n, "AGPRs": n, "ScratchSize": n, "Occupancy": n}} from
    -Rpass-analysis=kernel-resource-usage remarks."""
    out, cur = {}, None
    for ln in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", ln)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", ln)
        if m and cur is not None:
            cur[m.group(1).split()[0]] = int(m.group(2))
    return out


def check_resources(usage: dict) -> None:
    bad = []
    for name, u in usage.items():
        if "rollout_trace_kernel" in name:
            continue  # verification kernel: its per-step record stores may spill
        if u.get("ScratchSize", 0) != 0:
            bad.append(f"{name}: {u['ScratchSize']} bytes/lane of scratch (register spills)")
        if ("rollout_kernel" in name or "persistent_kernel" in name) and u.get("Occupancy", 0) < 2:
            bad.append(f"{name}: {u.get('VGPRs')} VGPRs + {u.get('AGPRs')} AGPRs, occupancy {u.get('Occupancy')} < 2")
    if not usage:
        bad.append("no kernel resource remarks were produced")
    if bad:
        raise RuntimeError("kernel resource check failed:\n" + "\n".join(bad))


# Host code only (the runtime: validation, tables, batching, the server's worker
# thread) under AddressSanitizer and UndefinedBehaviorSanitizer; device code is
# built as in the product library.  Load it with MPPI_LIB and clang's ASan
# runtime preloaded (sanitizer_runtime()).
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g", "-shared-libsan"]


def sanitizer_runtime() -> str:
    """clang's shared ASan runtime that the host-sanitizer build links against."""
    res = subprocess.run(["hipcc", "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        rd = subprocess.run(["hipcc", "--print-resource-dir"], capture_output=True, text=True).stdout.strip()
        path = os.path.join(rd, "lib", "linux", "libclang_rt.asan-x86_64.so")
    return path


def build(force: bool = True, verbose: bool = False, sanitize: bool = False) -> str:
    lib = LIB_SAN if sanitize else LIB
    if not force and os.path.exists(lib):
        mt = os.path.getmtime(lib)
        if all(os.path.getmtime(f) <= mt for f in SOURCES + HEADERS):
            return lib
    tmp = lib + ".tmp"
    extra = SAN_HOST if sanitize else []
    cmd = ["hipcc", *FLAGS, *extra, "-Rpass-analysis=kernel-resource-usage", *SOURCES, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("packed-fp32-ops", "kernel-resource-usage")
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines()
            if not any(n in ln for n in noise) and ln.strip() and not ln.startswith(" ") and ln.strip() != "^"]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    check_resources(resource_usage(res.stderr))
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
