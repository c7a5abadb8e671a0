"""Build the HIP library libpolymul.so for gfx950 (in-tree, no JIT cache).

    python -m paper_1609_01010_amd.build          # or build() from Python
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpolymul.so")
ARCH = os.environ.get("PM_OFFLOAD_ARCH", "gfx950")

# (source, extra defines): the kernel families are compiled once per value
# range of the prime (PM_LAZY=1: p < 2^30, PM_LAZY=0: p < 2^31)
SOURCES = [
    ("tables.hip", []),
    ("direct.hip", []),
    ("lds_conv.hip", ["-DPM_LAZY=0"]),
    ("lds_conv.hip", ["-DPM_LAZY=1"]),
    ("fourstep.hip", ["-DPM_LAZY=0"]),
    ("fourstep.hip", ["-DPM_LAZY=1"]),
    ("xform_kernels.hip", ["-DPM_LAZY=0"]),
    ("xform_kernels.hip", ["-DPM_LAZY=1"]),
    ("crt.hip", []),
    ("kronecker.hip", []),
    ("mixed.hip", []),
    ("dispatch.cpp", []),
    ("capi.cpp", []),
    ("batch.cpp", []),
    ("tune.cpp", []),
    ("mlp.hip", []),
    ("trace.cpp", []),
]

CFLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "--offload-arch=" + ARCH,
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _compile(item) -> str:
    src, defs = item
    path = os.path.join(CSRC, src)
    tag = "".join(d.replace("-D", ".").replace("=", "") for d in defs)
    obj = os.path.join(OBJ, src + tag + ".o")
    deps = [path] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(HERE, "..", "include", "polymul.h"))
    if os.path.exists(obj) and all(os.path.getmtime(obj) >= os.path.getmtime(d) for d in deps):
        return obj
    cmd = ["hipcc", "-x", "hip", *CFLAGS, *defs, "-c", path, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on " + src)
    os.replace(obj + ".tmp", obj)
    return obj


def build(force: bool = False, jobs: int | None = None) -> str:
    """Compile every source for gfx950 and link libpolymul.so; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    if force:
        for f in os.listdir(OBJ):
            os.remove(os.path.join(OBJ, f))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
