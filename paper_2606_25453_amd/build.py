"""Build the HIP library libozk.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libozk.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC, "-Wno-unused-result",
]


# compiled once per slice count (-DOZK_S1_P=p) so the kernels build in parallel
PER_P = {"s1_gemm_inst.hip"}
MAX_P = 8


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def units():
    """(source, object, extra flags) for every compilation."""
    out = []
    for src in sources():
        base = os.path.basename(src)[:-4]
        if os.path.basename(src) in PER_P:
            for p in range(1, MAX_P + 1):
                out.append((src, os.path.join(OBJDIR, "%s_p%d.o" % (base, p)), ["-DOZK_S1_P=%d" % p]))
        else:
            out.append((src, os.path.join(OBJDIR, base + ".o"), []))
    return out


def _compile(unit) -> str:
    src, obj, extra = unit
    subprocess.check_call([HIPCC, *FLAGS, *extra, "-c", src, "-o", obj])
    return obj


def build(verbose: bool = False) -> str:
    """Compile every kernel source and link libozk.so (always rebuilds)."""
    os.makedirs(OBJDIR, exist_ok=True)
    todo = units()
    # the longest compilations first
    todo.sort(key=lambda u: (os.path.basename(u[0]) not in PER_P, u[1]))
    with cf.ThreadPoolExecutor(max_workers=min(os.cpu_count() or 8, 16, len(todo))) as ex:
        objs = list(ex.map(_compile, todo))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
