"""Build liblbm.so (HIP, gfx950) in-tree with hipcc.

``python -m paper_2512_23116_amd.build`` compiles every ``csrc/*.hip`` into
``paper_2512_23116_amd/liblbm.so``.  Packed-FP32 instruction selection is
switched off (``-packed-fp32-ops``): the kernels rely on plain VALU FP32.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm.so")
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose=False, extra=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), *sources(),
           "-L/opt/rocm/lib", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


EXAMPLE_SRC = os.path.join(HERE, "examples", "forced_hit.c")
EXAMPLE = os.path.join(HERE, "examples", "forced_hit")


def build_examples(verbose=False):
    """Plain-C example linked against the in-tree liblbm.so (found next to the
    package at run time through an $ORIGIN-relative rpath)."""
    cc = os.environ.get("CC", "gcc")
    cmd = [cc, "-O2", "-std=c11", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"),
           EXAMPLE_SRC, "-L" + HERE, "-llbm", "-Wl,-rpath,$ORIGIN/..",
           "-Wl,-rpath-link,/opt/rocm/lib", "-o", EXAMPLE + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(EXAMPLE + ".tmp", EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
    build_examples(verbose=True)
