"""Sanitizer runs on the host (CPU only): the oracle compiled with
-fsanitize=address,undefined and driven over every entry point and boundary
kind (tests/sanitize/oracle_driver.c), and the host side of libase's C ABI
-- argument validation, workspace queries, batch packing -- compiled with
the host pass sanitized against launchers that do nothing
(tests/sanitize/api_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = os.path.join(HERE, "sanitize")


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-fopenmp", "-o", exe, os.path.join(SAN, "oracle_driver.c"), "-lm"],
                   check=True)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "2"})
    assert "0 failed" in out


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_c_abi_validation_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "api_asan")
    subprocess.run([_hipcc(), "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                    os.path.join(SAN, "api_driver.cpp"), "-o", exe],
                   check=True, capture_output=True)
    # the HIP runtime's own allocations outlive main: leak checking off here
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
    assert "0 failed" in out
