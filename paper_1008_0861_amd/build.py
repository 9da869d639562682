"""Build libasd.so (the gfx950 HIP library behind include/asd.h) in-tree.

    python -m paper_1008_0861_amd.build

Each source is compiled with hipcc for gfx950 only, then linked into
paper_1008_0861_amd/libasd.so.  Objects go to paper_1008_0861_amd/_build/.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libasd.so")
SOURCES = ["sweep.hip", "coef.hip", "explicit.hip", "util.hip", "adjoint.hip", "batch.hip", "capi.cpp",
           "graph.cpp", "adjoint_api.cpp", "batch_api.cpp", "bench_api.cpp", "noalloc.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-mcode-object-version=5",
    # never emit packed FP32 arithmetic (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]
# Per-source additions.  sweep.hip: gfx950 kernel-argument preloading of the
# sweep kernel's leading scalar arguments (the compiler preloads at most 14
# dwords; the kernel's argument list is laid out for that).
SOURCE_FLAGS = {"sweep.hip": ["-mllvm", "-amdgpu-kernarg-preload-count=16"]}


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC, "-x", "hip", *FLAGS, *SOURCE_FLAGS.get(src, []), "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, r.returncode, r.stdout + r.stderr, obj


def build(verbose=False):
    """Compile every source and link libasd.so; raises on failure."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = min(8, len(srcs))
    objs = []
    with ThreadPoolExecutor(jobs) as ex:
        for src, rc, out, obj in ex.map(_compile, srcs):
            # the host pass does not know the packed-fp32 feature: drop that warning
            msg = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip())
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{out}")
            if msg and verbose:
                print(msg, file=sys.stderr)
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
