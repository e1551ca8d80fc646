"""The CPU test suite again, with the library's host code (set-up and layout
builder, C-ABI argument checks, tune cache, network entry points) and the C
oracle built under AddressSanitizer + UndefinedBehaviorSanitizer.

The sanitized builds come from paper_2205_08909_amd.build_sanitized (rebuilt
here when older than their sources); a child interpreter preloads clang's
ASan runtime, selects them through MFCG_LIBRARY / MFCG_ORACLE_LIBRARY and
runs every other CPU test.  Any sanitizer report aborts the child, so the
test fails on it.  Leak checking is off: the interpreter itself keeps
allocations alive at exit.
"""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(target, sources):
    if not os.path.exists(target):
        return True
    t = os.path.getmtime(target)
    return any(os.path.getmtime(s) > t for s in sources)


def _sanitized_libs():
    from paper_2205_08909_amd import build_sanitized as bs
    csrc = os.path.join(ROOT, "paper_2205_08909_amd", "csrc")
    srcs = (glob.glob(os.path.join(csrc, "*")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
            + [bs.ORACLE_SRC])
    if _stale(bs.LIB, srcs) or _stale(bs.ORACLE_LIB, srcs):
        bs.build(verbose=False)
    return bs.LIB, bs.ORACLE_LIB, bs.runtime_library()


def _env(lib, olib, rt):
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "MFCG_LIBRARY": lib, "MFCG_ORACLE_LIBRARY": olib,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "PYTHONDONTWRITEBYTECODE": "1"})
    return env


def test_sanitized_libraries_are_the_ones_loaded():
    lib, olib, rt = _sanitized_libs()
    probe = ("from paper_2205_08909_amd import mfcg; from oracle import oracle; mfcg.lib(); oracle.lib(); "
             "maps = open('/proc/self/maps').read(); "
             "print(all(os.path.basename(p) in maps for p in (%r, %r, %r)))" % (lib, olib, rt))
    r = subprocess.run([sys.executable, "-c", "import os; " + probe], cwd=ROOT, env=_env(lib, olib, rt),
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("True"), r.stdout[-3000:]


def test_cpu_suite_under_host_sanitizers():
    lib, olib, rt = _sanitized_libs()
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        "tests", "--deselect", "tests/test_host_sanitizers.py"],
                       cwd=ROOT, env=_env(lib, olib, rt), stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=1200)
    tail = r.stdout[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stdout and "runtime error" not in r.stdout, tail
    assert " passed" in tail
