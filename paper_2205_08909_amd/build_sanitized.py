"""Host AddressSanitizer + UndefinedBehaviorSanitizer builds of the library's
host code and of the CPU oracle, for the CPU test suite.

    python -m paper_2205_08909_amd.build_sanitized

libmfcg_san.so: the host translation units (capi.hip, nn_capi.hip,
setup_host.cpp) recompiled with the sanitizers on their host pass only
(device code is never instrumented); every other object is the regular
build's.  liboracle_san.so: the oracle's C source built with clang and the
same sanitizers (without OpenMP).  Both link the shared ASan runtime, which
the process must preload (runtime_library() names it); tests select them
through MFCG_LIBRARY and MFCG_ORACLE_LIBRARY.
"""
import glob
import os
import subprocess
import sys

from paper_2205_08909_amd import build as base

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN_OBJDIR = os.path.join(ROOT, "_build", "objs_san")
LIB = os.path.join(HERE, "libmfcg_san.so")
ORACLE_SRC = os.path.join(ROOT, "oracle", "mfcg_oracle.c")
ORACLE_LIB = os.path.join(ROOT, "oracle", "liboracle_san.so")
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_SOURCES = ("capi.hip", "nn_capi.hip", "setup_host.cpp")

# each sanitizer flag is scoped to the host pass
SAN_HOST = []
for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-shared-libasan", "-g"):
    SAN_HOST += ["-Xarch_host", f]


def runtime_library():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not libs:
        raise RuntimeError("clang's shared ASan runtime is not installed")
    return libs[-1]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    msg = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"{cmd[0]} failed:\n{msg}")


def build(verbose=True):
    os.makedirs(SAN_OBJDIR, exist_ok=True)
    # the regular objects first (device code and the kernels' host stubs)
    base.build(verbose=False, incremental=True)
    objs = []
    for src in base.sources():
        name = os.path.basename(src)
        if name in HOST_SOURCES:
            out = os.path.join(SAN_OBJDIR, name + ".o")
            _run([base.HIPCC] + base.FLAGS + SAN_HOST + ["-c", "-o", out, src], verbose)
            objs.append(out)
        else:
            objs.append(base._obj(src))
    rt_dir = os.path.dirname(runtime_library())
    _run([base.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
         + ["-L" + rt_dir, "-lclang_rt.asan-x86_64", "-Wl,-rpath," + rt_dir], verbose)
    os.replace(LIB + ".tmp", LIB)
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-fno-omit-frame-pointer", "-shared-libasan", "-Wno-unknown-pragmas", "-shared", "-fPIC", "-std=c11",
          "-o", ORACLE_LIB + ".tmp", ORACLE_SRC, "-lm", "-Wl,-rpath," + rt_dir], verbose)
    os.replace(ORACLE_LIB + ".tmp", ORACLE_LIB)
    return LIB, ORACLE_LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv[1:])
