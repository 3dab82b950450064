"""Build the lbm3d HIP library for gfx950 in-tree (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm3d.so")
SOURCES = ["lbm3d_device.hip", "lbm3d_layout.cpp", "lbm3d_api.cpp", "lbm3d_batch.cpp", "lbm3d_server.cpp",
           "lbm3d_tune.cpp", "lbm3d_probe.hip", "lbm3d_stability.cpp"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

# gfx950 only; packed FP32 instructions are switched off for all device code
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    # contract a*b+c only within one expression, so that the same source
    # rounds the same way in every kernel it is inlined into
    "-ffp-contract=on",
]


def _objects(jobs):
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, "_build", "%08x" % (hash(tuple(FLAGS)) & 0xffffffff), src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmd = [os.path.join(ROCM, "bin", "hipcc")] + lang + FLAGS + ["-c", path, "-o", obj]
        jobs.append(subprocess.Popen(cmd))
        objs.append(obj)
    return objs


def build(defines=(), out=None) -> str:
    """Compile and link the library; `defines` are extra -D tuning knobs and
    `out` an alternative output path (both for tuning builds)."""
    global FLAGS
    base_flags = FLAGS
    FLAGS = FLAGS + ["-D" + d for d in defines]
    try:
        return _build(out or LIB)
    finally:
        FLAGS = base_flags


def _build(lib) -> str:
    jobs = []
    objs = _objects(jobs)
    rc = [j.wait() for j in jobs]
    if any(rc):
        raise RuntimeError("hipcc failed")
    tmp = lib + ".tmp"
    cmd = [os.path.join(ROCM, "bin", "hipcc"), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build())
    sys.exit(0)
