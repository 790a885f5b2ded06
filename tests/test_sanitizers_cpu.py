"""Host code under the address and undefined-behaviour sanitizers (CPU only):
the C-ABI's argument checks, camera composition and early error returns
(capi.cpp linked with kernel-launch stand-ins, driven by a C program), and
the oracle's C steps on small inputs (built with the sanitizers and loaded
into a Python process with the address sanitizer preloaded)."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2411_16680_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_capi_host_code_under_sanitizers(tmp_path):
    hip = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    _run(["g++", "-std=c++17", *SAN, *hip, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
          os.path.join(CSRC, "capi.cpp"), "-o", str(tmp_path / "capi.o")])
    _run(["g++", "-std=c++17", *SAN, *hip, "-I", CSRC, "-c", os.path.join(HERE, "host_stubs.cpp"),
          "-o", str(tmp_path / "stubs.o")])
    _run(["gcc", "-std=c11", *SAN, "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(HERE, "capi_driver.c"), "-o", str(tmp_path / "drv.o")])
    exe = str(tmp_path / "drv")
    _run(["g++", *SAN, str(tmp_path / "drv.o"), str(tmp_path / "capi.o"), str(tmp_path / "stubs.o"),
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=ENV, timeout=120)
    assert " 0 failures" in r.stdout, r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]


def test_oracle_under_sanitizers(tmp_path):
    so = str(tmp_path / "liboracle_san.so")
    _run(["gcc", "-std=c11", *SAN, "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
          os.path.join(ROOT, "oracle", "quark_oracle.c"), "-o", so, "-lm"])
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    env = dict(ENV, LD_PRELOAD=asan, OMP_NUM_THREADS="2")
    r = _run([sys.executable, os.path.join(HERE, "oracle_exercise.py"), so], env=env, timeout=300)
    assert "oracle ok" in r.stdout, (r.stdout, r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
