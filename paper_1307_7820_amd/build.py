"""Build libnf.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1307_7820_amd.build          # build
    python -m paper_1307_7820_amd.build --print  # show the command

The shared library lands next to this file; ``nf.py`` loads it from there.
"""

from __future__ import annotations

import os
import shlex
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnf.so")

SOURCES = ["nf_kernels.hip", "nf_traceback.hip", "nf_plain.hip", "nf_noalloc.hip", "nf_measure.hip", "nf_runtime.cpp",
           "nf_api.cpp", "nf_serve.cpp"]
HEADERS = ["nf_internal.h", "nf_runtime.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-result",
    # no packed fp32 instructions in any device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE,
    "-I" + CSRC,
    "-pthread",
]


def command(out: str = LIB):
    return [HIPCC, *FLAGS, *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


# The paper's serial CPU algorithms (include/nf_serial.h): plain host C++,
# a library of its own that libnf.so never calls.
SERIAL_LIB = os.path.join(HERE, "libnf_serial.so")
SERIAL_FLAGS = ["-O3", "-march=x86-64-v3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-Wall", "-I" + INCLUDE]


def serial_command(out: str = SERIAL_LIB):
    return [os.environ.get("CXX", "g++"), *SERIAL_FLAGS, os.path.join(CSRC, "nf_serial.cpp"), "-o", out]


def build_serial(verbose: bool = False) -> str:
    """Compile nf_serial.cpp into libnf_serial.so (always recompiles)."""
    tmp = SERIAL_LIB + ".tmp%d" % os.getpid()
    cmd = serial_command(tmp)
    if verbose:
        print(" ".join(shlex.quote(c) for c in cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SERIAL_LIB)
    return SERIAL_LIB


def build(verbose: bool = False) -> str:
    """Compile every source into libnf.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(shlex.quote(c) for c in cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def up_to_date() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(INCLUDE, "nf.h")]
    return all(os.path.getmtime(d) <= t for d in deps)


if __name__ == "__main__":
    if "--print" in sys.argv:
        print(" ".join(shlex.quote(c) for c in command()))
        print(" ".join(shlex.quote(c) for c in serial_command()))
    else:
        print(build(verbose=True))
        print(build_serial(verbose=True))
