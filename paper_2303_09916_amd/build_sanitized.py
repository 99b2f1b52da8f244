"""Host-sanitizer build (CPU only): the library with AddressSanitizer and UBSan
in its host code (input validation, ligand packing, the C-ABI entry points, the
serving scheduler) and the FP64 oracle with both sanitizers, then the CPU test
suite (-m "not gpu") run against them.

    python paper_2303_09916_amd/build_sanitized.py [--no-tests]

Builds _build_san/libdsdp_san.so and _build_san/liboracle_san.so (clang, shared
ASan runtime) and runs pytest with that runtime preloaded, DSDP_LIB and
DSDP_ORACLE_LIB pointing at the sanitized builds.  The device code is built as
usual; sanitizers act on host code only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(ROOT, "_build_san")
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
DEVICE_SOURCES = ["grid_build.hip", "search.hip", "site.hip", "probe.hip"]
HOST_SOURCES = ["dsdp_abi.cpp", "dsdp_sched.cpp"]
SAN = ["address", "undefined"]


def run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build():
    os.makedirs(OUT, exist_ok=True)
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-w", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for s in DEVICE_SOURCES:
        o = os.path.join(OUT, s + ".o")
        run([HIPCC, "-c"] + common + [os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    host_san = []
    for k in SAN:
        host_san += ["-Xarch_host", "-fsanitize=" + k]
    host_san += ["-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    for s in HOST_SOURCES:
        o = os.path.join(OUT, s + ".o")
        run([HIPCC, "-c"] + common + host_san + [os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    lib = os.path.join(OUT, "libdsdp_san.so")
    link_san = ["-fsanitize=" + ",".join(SAN), "-shared-libasan"]
    run([CLANG + "++", "-shared", "-fPIC"] + link_san + objs +
        ["-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", lib])
    olib = os.path.join(OUT, "liboracle_san.so")
    run([CLANG, "-std=c11", "-O1", "-g", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-fno-omit-frame-pointer",
         "-fno-sanitize-recover=all"] + link_san + [os.path.join(ROOT, "oracle", "dsdp_oracle.c"), "-o", olib, "-lm"])
    return lib, olib


def run_tests(lib, olib):
    rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], check=True, capture_output=True,
                        text=True).stdout.strip()
    if not os.path.exists(rt):
        raise SystemExit(f"ASan runtime not found: {rt}")
    env = dict(os.environ, LD_PRELOAD=rt, DSDP_LIB=lib, DSDP_ORACLE_LIB=olib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests")], env=env, cwd=ROOT)
    return r.returncode


if __name__ == "__main__":
    lib, olib = build()
    if "--no-tests" not in sys.argv:
        sys.exit(run_tests(lib, olib))
