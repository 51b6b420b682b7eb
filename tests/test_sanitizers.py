"""CPU sanitizer job: the oracle (oracle.c) and the library's host code (argument validation,
workspace planning, the C ABI's bookkeeping) built with AddressSanitizer and
UndefinedBehaviorSanitizer, and the oracle's pins plus the host-side ABI tests run against those
builds in a child process with the sanitizer runtime preloaded; any report fails the run.

Opt-in (it rebuilds the HIP library, several minutes): BRI_SANITIZE=1 python -m pytest
tests/test_sanitizers.py.  The device code is compiled as usual."""

import glob
import os
import subprocess
import sys

import pytest

from tests.conftest import ROOT

pytestmark = pytest.mark.sanitize


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_oracle_and_host_code_under_asan_ubsan(tmp_path):
    if os.environ.get("BRI_SANITIZE") != "1":
        pytest.skip("opt-in: set BRI_SANITIZE=1")
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no clang sanitizer runtime")
    sys.path.insert(0, ROOT)
    import oracle
    from paper_1701_00726_amd import build as hipbuild

    olib = oracle.build(sanitize_to=str(tmp_path / "liboracle_san.so"))
    blib = hipbuild.build(sanitize_to=str(tmp_path / "libbrillouin_san.so"))
    env = dict(os.environ, LD_PRELOAD=rt, ORACLE_LIB=olib, BRI_LIB=blib, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py"))) + [
        os.path.join(ROOT, "tests", "test_abi.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu and not slow", "-p",
                        "no:cacheprovider", *files], cwd=ROOT, env=env, capture_output=True, text=True, timeout=3600)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
