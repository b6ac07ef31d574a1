"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The oracle (oracle.cpp) is rebuilt with g++ and both sanitizers and the
  oracle pin suite runs against it.
* libmacsplat is rebuilt with both sanitizers on its host pass only (every
  flag behind -Xarch_host; the device code is built as usual) and the CPU
  tests of the C ABI run against it: every argument check, rejection path
  and symbol lookup of api.cpp, with no GPU in reach.

Each run is a child process with the sanitizer runtime preloaded (Python
itself is not instrumented), halting on the first report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "PYTHONDONTWRITEBYTECODE": "1"}


def _runtime(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def _run_child(code: str, preload: str, timeout: int = 600):
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=preload)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=timeout)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    return out


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime(["g++", "-print-file-name=libasan.so"])
    if asan is None:
        pytest.skip("g++ has no AddressSanitizer runtime here")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-fPIC", "-shared", os.path.join(ROOT, "oracle", "oracle.cpp"), "-o", lib], check=True)
    code = f"""
import ctypes, sys
import pytest
import oracle.oracle as oo
oo._lib = ctypes.CDLL({lib!r})
oo._declare(oo._lib)
oo.build = lambda force=True: {lib!r}
sys.exit(pytest.main(["-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", "tests/test_oracle_pins.py",
                      "tests/test_cull_bound.py"]))
"""
    out = _run_child(code, asan)
    assert " passed" in out, out[-3000:]


def test_library_host_validation_under_asan_and_ubsan(tmp_path):
    clang_rt = _runtime(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"])
    if clang_rt is None:
        pytest.skip("clang has no shared AddressSanitizer runtime here")
    from paper_2412_09723_amd import build
    host = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
              "-g"):
        host += ["-Xarch_host", f]
    lib = build.build(out=str(tmp_path / "libmacsplat_san.so"), obj_dir=str(tmp_path / "obj"), host_flags=host,
                      link_flags=["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                                  "-shared-libsan"])
    code = f"""
import sys
import pytest
import paper_2412_09723_amd._lib as L
L.LIB_PATH = {lib!r}
lib = L.load()
assert lib._name == {lib!r}
sys.exit(pytest.main(["-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", "tests/test_abi.py"]))
"""
    out = _run_child(code, clang_rt)
    assert " passed" in out, out[-3000:]
