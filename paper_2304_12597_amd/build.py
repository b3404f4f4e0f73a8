"""Build libparadiag.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libparadiag.so")
ARCH = os.environ.get("PD_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC",
         # packed FP32 instructions are disabled for every HIP source
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # multiply-adds are fused per source expression only, so a device
         # function rounds the same way in every kernel it is inlined into
         # (single-problem and batched launches agree bit for bit)
         "-ffp-contract=on",
         "-Wno-unused-result"]


def source_hash() -> str:
    """sha256 over the native sources and build.py itself: a recorded
    hardware-counter reading is valid only for the kernels it was taken on."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                   if f.endswith((".hip", ".h")))
    for path in files + [os.path.abspath(__file__)]:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    cmd = ["hipcc"] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(jobs: int = 8) -> str:
    """Compile every csrc/*.hip and link libparadiag.so (always rebuilds)."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    # roctx (host ranges for profilers) from the ROCm install, found at run
    # time through the rpath
    r = subprocess.run(["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs +
                       ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
