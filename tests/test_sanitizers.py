"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* the plan compiler and the host part of ingest (csrc/plan.cpp,
  csrc/ingest.cpp), built with g++ into tests/sanitize/host_driver.cpp;
* the oracle's C code (oracle/oracle.c), built with gcc into
  tests/sanitize/oracle_driver.c, and loaded by the oracle's own tests with
  libasan preloaded (ORACLE_SANITIZE=1 selects the sanitized build).

No GPU code is built here: the HIP kernels are outside what these tools see.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
       "-fno-sanitize-recover=undefined"]


def _env():
    env = dict(os.environ)
    # leak reports would flag the interpreter's own arenas; keep the memory errors
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not installed")


def _run(cmd, timeout, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, **kw)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


def test_host_driver(tmp_path):
    _need("g++")
    exe = str(tmp_path / "host_driver")
    csrc = os.path.join(ROOT, "paper_2004_02369_amd", "csrc")
    _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
          os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
          os.path.join(csrc, "plan.cpp"), os.path.join(csrc, "ingest.cpp"), "-o", exe], 300)
    assert "host driver ok" in _run([exe], 300, env=_env())


def test_oracle_driver(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c11", *SAN, "-pthread", os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
          "-o", exe], 300)
    assert "oracle driver ok" in _run([exe], 300, env=_env())


def test_oracle_tests_under_asan():
    _need("gcc")
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
        if not os.path.isabs(p) or not os.path.exists(p):
            pytest.skip(f"{name} not found")
        libs.append(p)
    env = _env()
    env["ORACLE_SANITIZE"] = "1"
    env["LD_PRELOAD"] = ":".join(libs)
    # the star row over 5 vertices takes minutes under the sanitizers; its
    # 4-vertex case runs the same code
    _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
          "tests/test_oracle.py", "tests/test_oracle_mni.py", "tests/test_motifs.py",
          "--deselect", "tests/test_oracle.py::test_star_row_invariant[5]"], 600, env=env, cwd=ROOT)
