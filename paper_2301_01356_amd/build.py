"""Build the native parts in-tree.

* ``libfastbcc.so``  -- the HIP library (gfx950 only) behind ``include/fastbcc.h``.
* ``gen/libgraphgen.so`` -- the seeded host-side graph generators.

Run ``python -m paper_2301_01356_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
HIP_SOURCES = [os.path.join(PKG, "csrc", f) for f in ("fastbcc.hip", "small.hip")]
LIB = os.path.join(PKG, "libfastbcc.so")
GEN_SRC = os.path.join(PKG, "gen", "graphgen.cpp")
GEN_LIB = os.path.join(PKG, "gen", "libgraphgen.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-shared",
    "-fPIC",
    "-fvisibility=hidden",
    "-Wall",
    "-Wno-unused-function",
    # packed fp32 ops are kept out of every code object built here
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_gen() -> str:
    _run(["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC", GEN_SRC, "-o", GEN_LIB + ".tmp"])
    os.replace(GEN_LIB + ".tmp", GEN_LIB)
    return GEN_LIB


def build_native() -> str:
    inc = os.path.join(ROOT, "include")
    _run([HIPCC, *HIP_FLAGS, "-I", inc, *HIP_SOURCES, "-o", LIB + ".tmp"])
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_all() -> None:
    build_gen()
    build_native()


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    {"gen": build_gen, "native": build_native, "all": build_all}[what]()
