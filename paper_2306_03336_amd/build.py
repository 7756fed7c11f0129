"""Build libdtb.so in-tree with hipcc for gfx950.

    python -m paper_2306_03336_amd.build        # or build() from Python

Objects go to ``_build/`` at the repository root; the shared library is
written next to this file as ``libdtb.so``.  Every compile line carries
``-Xclang -target-feature -Xclang -packed-fp32-ops`` (no packed FP32
instructions are generated) and ``-ffp-contract=off`` (no multiply-add is
fused unless the source asks for it).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_PATH = os.path.join(HERE, "libdtb.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]

_HIP = ["-x", "hip", f"--offload-arch={ARCH}"]
# Largest translation units first so the parallel build finishes sooner.
SOURCES = [(f"dtb_inst_{n}.hip", _HIP) for n in ("f32_r28", "f32_r24", "batch", "f64_r24", "f64c4_r12", "f64w4_r24", "f32_r16",
                                                 "f64_r16", "f32_r8", "f64_r8", "box_f64_r8",
                                                 "box_f32_r16", "3d")] + [
    ("dtb_kernels.hip", _HIP),
    ("dtb_probe.hip", _HIP),
    ("dtb_noalloc.hip", _HIP),
    ("dtb_plan.cpp", []),
    ("dtb_api.cpp", ["-D__HIP_PLATFORM_AMD__"]),
]


def kernel_source_hash() -> str:
    """SHA-256 over the device sources (csrc/*.h, csrc/*.hip): measurements recorded for one
    version of the kernels (HBM traffic, accuracy) are reported only while this still matches."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def _up_to_date(src: str, obj: str) -> bool:
    """With DTB_INCREMENTAL=1: the object is newer than its source and every header."""
    if os.environ.get("DTB_INCREMENTAL") != "1" or not os.path.exists(obj):
        return False
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")] + \
        [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in deps)


def _compile(src: str, extra: list) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    if _up_to_date(src, obj):
        return obj
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
