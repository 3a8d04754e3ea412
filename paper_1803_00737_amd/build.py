"""Build the HIP library ``libdwtfuse.so`` in-tree for gfx950 with hipcc.

    python -m paper_1803_00737_amd.build
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(PKG, "libdwtfuse.so")
BUILD_DIR = os.path.join(ROOT, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SOURCES = ["dwt_fuse_api.cpp", "fuse_kernels.hip", "adjoint_kernels.hip", "multipass_kernels.hip", "codec_kernels.hip",
           "quality_kernels.hip", "static_scratch.hip"]
HEADERS = [os.path.join(CSRC, "fuse_internal.h"), os.path.join(CSRC, "fuse_math.h"), os.path.join(INCLUDE, "dwt_fuse.h")]

# -packed-fp32-ops: keep the compiler from forming packed FP32 arithmetic.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                # loadable by the HIP runtime bundled with PyTorch as well as /opt/rocm
                "-mcode-object-version=5"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm toolchain required to build the HIP library)")


def build_id() -> str:
    h = hashlib.sha1()
    for f in [os.path.join(CSRC, s) for s in SOURCES] + HEADERS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def build(verbose: bool = False, arch: str = "gfx950") -> str:
    """Compile every source for ``arch`` and link the shared library (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    bid = build_id()
    # Only the C ABI of include/dwt_fuse.h is exported (dwt_fuse_api.cpp
    # includes the header with default visibility); everything else is hidden.
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-fvisibility=hidden", "-I", INCLUDE, "-I", CSRC,
              '-DDWT_FUSE_BUILD_ID="%s"' % bid]

    def compile_one(src):
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD_DIR, src + ".o")
        if src.endswith(".hip"):
            cmd = [cc, "--offload-arch=" + arch, "-x", "hip"] + DEVICE_FLAGS + common + ["-c", path, "-o", obj]
        else:
            cmd = [cc, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include")] + common + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s%s" % (src, r.stdout, r.stderr))
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = [cc, "--offload-arch=" + arch, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB_PATH)
    with open(os.path.join(PKG, "libdwtfuse.buildid"), "w") as f:
        f.write(bid + "\n")
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
