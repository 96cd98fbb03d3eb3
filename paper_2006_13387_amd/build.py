"""Build libmsp.so (hand-written HIP for gfx950) in-tree with hipcc.

    python -m paper_2006_13387_amd.build

Every call recompiles all sources.  The library lands next to this file so
that it travels with the source tree.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmsp.so")

SOURCES = ["k_vec.hip", "k_local.hip", "k_coarse.hip", "k_topo.hip", "k_3d.hip",
           "k_coarse3d.hip", "k_ee2d.hip",
           "noalloc.hip", "runtime.cpp", "elements.cpp"]

ARCH = os.environ.get("MSP_OFFLOAD_ARCH", "gfx950")
# packed FP32 instructions are disabled for all device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable", "-Wno-unused-but-set-variable"]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found (ROCm toolchain required)")
    return path


def _compile(src, obj):
    cmd = [hipcc(), *COMMON, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src),
           "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{res.stderr}")
    # hipcc's host pass warns that it does not know the device feature flag
    msgs = [l for l in res.stderr.splitlines()
            if l.strip() and "packed-fp32-ops" not in l]
    return src, msgs


def build(verbose=True):
    """Compile every source and link libmsp.so; returns the library path."""
    with tempfile.TemporaryDirectory(prefix="msp_build_") as tmp:
        objs = [os.path.join(tmp, s + ".o") for s in SOURCES]
        with concurrent.futures.ThreadPoolExecutor(max_workers=7) as ex:
            futs = [ex.submit(_compile, s, o) for s, o in zip(SOURCES, objs)]
            for f in futs:
                src, msgs = f.result()
                if verbose and msgs:
                    print(f"[build] {src}:\n  " + "\n  ".join(msgs[:20]))
        out_tmp = LIB + ".tmp"
        cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs,
               "-o", out_tmp]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"linking libmsp.so failed:\n{res.stderr}")
        os.replace(out_tmp, LIB)
    if verbose:
        print(f"[build] {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
