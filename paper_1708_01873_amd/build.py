"""Compile libbitrev.so (HIP, gfx950) in-tree.

``python -m paper_1708_01873_amd.build`` or ``build()``: every ``csrc/*.hip``
file is compiled with hipcc in parallel and linked into
``paper_1708_01873_amd/libbitrev.so``.  Always recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(PKG, "_build")
LIBRARY = os.path.join(PKG, "libbitrev.so")
ARCH = os.environ.get("BITREV_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-fno-strict-aliasing",
    # Keep the compiler from emitting packed FP32 instructions (the fused FFT
    # levels are the only float arithmetic; they must not use them).
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-I", CSRC,
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: libbitrev needs ROCm to build")
    return path


# The compiler's per-kernel resource remarks (registers, scratch, LDS).
RESOURCE_FLAG = "-Rpass-analysis=kernel-resource-usage"
RESOURCES = os.path.join(BUILD_DIR, "kernel_resources.txt")
_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|LDS Size \[bytes/block\]):\s+(\S+)")


def parse_resources(text: str) -> list[dict]:
    """Kernels and their resource figures from hipcc's resource remarks."""
    kernels: list[dict] = []
    for line in text.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1).split(" [")[0], m.group(2)
        if key == "Function Name":
            kernels.append({"name": val})
        elif kernels:
            kernels[-1][key] = int(val) if val.isdigit() else val
    return kernels


def _compile(src: str, extra: list[str]) -> tuple[str, list[dict]]:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [hipcc()] + HIPCC_FLAGS + [RESOURCE_FLAG] + extra + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), p.stderr))
    return obj, parse_resources(p.stderr)


def build(extra_flags: list[str] | None = None, jobs: int | None = None) -> str:
    """Compile every csrc/*.hip for gfx950 and link libbitrev.so."""
    extra = list(extra_flags or [])
    os.makedirs(BUILD_DIR, exist_ok=True)
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(len(sources), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, extra), sources))
    objs = [o for o, _ in results]
    kernels = [k for _, ks in results for k in ks]
    with open(RESOURCES, "w") as f:
        f.write("# kernel  VGPRs  AGPRs  scratch-bytes/lane  waves/SIMD  LDS-bytes/block\n")
        for k in sorted(kernels, key=lambda k: k["name"]):
            f.write("%s %s %s %s %s %s\n" % (k["name"], k.get("VGPRs"), k.get("AGPRs"),
                                           k.get("ScratchSize"), k.get("Occupancy"),
                                           k.get("LDS Size")))
    # every kernel keeps its working set in registers and LDS: a kernel that
    # spills to scratch memory is a build error, not a silent slowdown
    spills = [k["name"] for k in kernels if k.get("ScratchSize", 0) != 0]
    if spills:
        raise RuntimeError("kernels using scratch memory:\n  " + "\n  ".join(spills))
    tmp = LIBRARY + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), p.stderr))
    os.replace(tmp, LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    print(build(sys.argv[1:]))
