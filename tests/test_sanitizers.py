"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The pass planner (csrc/planner.cpp, host C++ with no HIP in it) is built
  with both sanitizers together with tests/planner_check.cpp, which plans
  random diagrams under many settings and checks every plan (each step once,
  admissible in its pass, non-commuting steps in order, the same result for
  M <= 14); any out-of-bounds access or undefined behaviour aborts it.
* The oracle (oracle/oracle.c) is built with both sanitizers and the pin
  tests run against that build (QSIM_ORACLE_LIB) in a child process with the
  ASan runtime preloaded.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _tool(name):
    path = shutil.which(name)
    if path is None:
        pytest.skip(f"{name} not found")
    return path


def _libasan():
    r = subprocess.run([_tool("gcc"), "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("gcc's ASan runtime not found")
    return path


def test_planner_under_sanitizers(tmp_path):
    exe = tmp_path / "planner_check"
    r = subprocess.run([_tool("g++"), "-std=c++17", *SAN, "-fno-sanitize-recover=all", "-pthread",
                        os.path.join(ROOT, "paper_quant_ph_0308158_amd", "csrc", "planner.cpp"),
                        os.path.join(ROOT, "tests", "planner_check.cpp"), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
                            "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "planner ok" in r.stdout


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    r = subprocess.run([_tool("gcc"), "-std=c11", "-fPIC", "-shared", "-fopenmp", *SAN,
                        "-fno-sanitize-recover=undefined", "-o", str(lib),
                        os.path.join(ROOT, "oracle", "oracle.c")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = {**os.environ, "LD_PRELOAD": _libasan(), "QSIM_ORACLE_LIB": str(lib),
           "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}
    # the child loads the sanitized build, not liboracle.so
    r = subprocess.run([sys.executable, "-c", "import oracle; oracle._load(); print(oracle.library_path())"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == str(lib), r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-x",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout
