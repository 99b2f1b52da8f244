"""Build libdsdp.so (HIP kernels for gfx950 + the C-ABI host code) in-tree with hipcc,
and the plain C client of its ABI that the tests run (tests/c_client)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdsdp.so")
SOURCES = ["grid_build.hip", "search.hip", "site.hip", "probe.hip", "dsdp_abi.cpp", "dsdp_sched.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose=False, extra=()):
    tmp = LIB + ".tmp"
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [HIPCC] + FLAGS + list(extra) + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_c_client(verbose=False):
    """tests/c_client: a C11 program that uses the library through include/dsdp.h
    and the HIP runtime only (gcc, no hipcc, no device code of its own)."""
    exe = os.path.join(ROOT, "tests", "c_client")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
           os.path.join(ROOT, "tests", "c_client.c"), "-o", exe + ".tmp",
           "-L", HERE, "-ldsdp", "-Wl,-rpath,$ORIGIN/../paper_2303_09916_amd",
           "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(exe + ".tmp", exe)
    return exe


if __name__ == "__main__":
    build(verbose=True, extra=[a for a in sys.argv[1:] if a != "-v"])
