"""Build libfhesnn.so (HIP kernels for gfx950 + host C++ + the C ABI) in-tree.

    python -m paper_2309_09025_amd.build

Cross-compiles without a GPU; the result sits next to this file and is what
the Python binding loads.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfhesnn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["host_keys.cpp", "capi.cpp", "pbs.hip", "linear.hip", "noalloc.hip", "ceiling.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # exact-arithmetic code: never contract a*b+c behind the source's back
    "-ffp-contract=off",
    # no packed fp32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _obj(src: str, outdir: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(outdir, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    subprocess.check_call([HIPCC, *FLAGS, *lang, "-c", path, "-o", obj])
    return obj


def build(verbose: bool = True) -> str:
    """Compile every source and link the shared library (always rebuilds)."""
    with tempfile.TemporaryDirectory(prefix="fhesnn_build_") as tmp:
        objs = [_obj(s, tmp) for s in SOURCES]
        out = LIB + ".tmp"
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out,
                               *objs, "-lpthread"])
        os.replace(out, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


C_CLIENT_SRC = os.path.join(ROOT, "tests", "c_abi_roundtrip.c")
C_CLIENT = os.path.join(ROOT, "tests", "c_abi_roundtrip")


def build_c_client(verbose: bool = True) -> str:
    """Compile the plain-C client of the library (include/fhesnn.h + the HIP
    runtime only) that a GPU test runs; it finds libfhesnn.so by rpath."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    out = C_CLIENT + ".tmp"
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-Wall", "-Wextra",
                           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(rocm, "include"), C_CLIENT_SRC, "-o", out,
                           "-L", HERE, "-lfhesnn", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
                           "-Wl,-rpath," + HERE, "-Wl,-rpath,$ORIGIN/../paper_2309_09025_amd"])
    os.replace(out, C_CLIENT)
    if verbose:
        print(f"built {C_CLIENT}", file=sys.stderr)
    return C_CLIENT


if __name__ == "__main__":
    build()
    build_c_client()
