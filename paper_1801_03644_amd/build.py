"""Build step for the package's native libraries (in-tree, for gfx950).

* ``lib/libmdrq.so``         the C-ABI range-query library: HIP kernels + host runtime,
                             compiled with hipcc for gfx950.
* ``lib/libmdrq_datagen.so`` the seeded input generator (plain C, gcc).

Run ``python -m paper_1801_03644_amd.build`` or call :func:`build_all`.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "lib")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(LIB, "obj")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# gfx950 only.  Packed-FP32 VALU forms are switched off for all device code; denormals
# are kept (float comparisons must stay exact for subnormal inputs).
HIP_FLAGS = [
    "-std=c++17", "-O3", "--offload-arch=gfx950", "-fPIC", "-Wall",
    "-fno-gpu-flush-denormals-to-zero", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]

DATAGEN_SRC = os.path.join(HERE, "datagen", "datagen.c")
DATAGEN_LIB = os.path.join(LIB, "libmdrq_datagen.so")
MDRQ_LIB = os.path.join(LIB, "libmdrq.so")


def _sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def build_datagen() -> str:
    os.makedirs(LIB, exist_ok=True)
    tmp = DATAGEN_LIB + ".tmp"
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-fno-fast-math", "-fPIC", "-shared",
                           "-Wall", "-o", tmp, DATAGEN_SRC, "-lm", "-lpthread"])
    os.replace(tmp, DATAGEN_LIB)
    return DATAGEN_LIB


# Per-file additions.  The shared-scan kernels add to their LDS counts from one lane
# with a wave-uniform value; the compiler's atomic optimizer would wrap each such add
# in a wave reduction that does nothing here.
FILE_FLAGS = {"batch.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]}


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *HIP_FLAGS, *FILE_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    subprocess.check_call(cmd)
    return obj


def build_mdrq(jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = _sources()
    if not srcs:
        raise RuntimeError("no HIP sources")
    jobs = jobs or min(16, max(1, os.cpu_count() or 1), len(srcs))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = MDRQ_LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
                           "-lpthread"])
    os.replace(tmp, MDRQ_LIB)
    return MDRQ_LIB


def build_all() -> None:
    build_datagen()
    build_mdrq()


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    {"all": build_all, "datagen": build_datagen, "mdrq": build_mdrq}[what]()
