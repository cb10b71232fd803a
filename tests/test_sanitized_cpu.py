"""The oracle and the library's host code (argument checks, workspace and
plan bookkeeping, the C ABI) built with AddressSanitizer and
UndefinedBehaviorSanitizer, and the CPU tests of the C ABI and of the oracle
run against those builds in a child Python with the sanitizer runtime
preloaded. Device code is compiled as usual (there is no GPU sanitizer run);
the builds are redone only when a source is newer than them."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "paper_2301_03636_amd", "_build_san")
RT = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
CHILD_TESTS = ["tests/test_abi_cpu.py", "tests/test_oracle_features.py",
               "tests/test_oracle_model.py", "tests/test_oracle_pins.py",
               "tests/test_oracle_lowering.py", "tests/test_oracle_variants.py",
               "tests/test_oracle_dataflow.py"]


def _stale(target, sources):
    return not os.path.exists(target) or os.path.getmtime(target) < max(
        os.path.getmtime(s) for s in sources)


@pytest.mark.skipif(not RT, reason="no clang sanitizer runtime in this ROCm install")
def test_abi_and_oracle_tests_under_asan_ubsan():
    sys.path.insert(0, ROOT)
    from paper_2301_03636_amd import build
    import oracle
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "libadvisor_san.so")
    olib = os.path.join(OUT, "liboracle_san.so")
    srcs = (glob.glob(os.path.join(ROOT, "paper_2301_03636_amd", "csrc", "*")) +
            glob.glob(os.path.join(ROOT, "include", "*.h")))
    if _stale(lib, srcs):
        build.build(out=lib, sanitize=True)
    if _stale(olib, [os.path.join(ROOT, "oracle", "oracle.c")]):
        oracle.build_sanitized(olib)
    env = dict(os.environ, LD_PRELOAD=RT[-1], ADVISOR_LIBRARY=lib, ORACLE_LIBRARY=olib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the child loads the sanitized builds, not the in-tree ones
    probe = ("import oracle, paper_2301_03636_amd as a; a._lib.lib(); oracle._load();"
             "m = open('/proc/self/maps').read();"
             "assert 'libadvisor_san.so' in m and 'liboracle_san.so' in m, 'not loaded';"
             "assert 'libclang_rt.asan' in m")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *CHILD_TESTS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    print(r.stdout[-800:])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
