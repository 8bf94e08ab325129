"""The CPU oracle and the library's host-side partition code built with the
host address and undefined-behaviour sanitizers and run over their entry
points (tests/hostsim/oracle_sanitize.c, tests/hostsim/partition_sanitize.cpp):
no sanitizer report, no unexpected status, partition counts equal to the
oracle's.  The buffers the library keeps per device until exit are the only
suppressed leaks (tests/hostsim/lsan_device_caches.supp)."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM = os.path.join(ROOT, "tests", "hostsim")
CSRC = os.path.join(ROOT, "paper_1905_03525_amd", "csrc")
ORACLE_C = os.path.join(ROOT, "oracle", "rmat_oracle.c")
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
       "-ffp-contract=off", "-pthread"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           LSAN_OPTIONS="suppressions=" + os.path.join(SIM, "lsan_device_caches.supp"))


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.run(["gcc", "-std=c11", *SAN, "-Wall", "-Wno-unused-function", ORACLE_C,
                    os.path.join(SIM, "oracle_sanitize.c"), "-o", exe, "-lm"], check=True, capture_output=True,
                   text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 unexpected statuses" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr


def test_partition_host_code_under_sanitizers(tmp_path):
    _need("gcc")
    _need("g++")
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "partition_sanitize")
    subprocess.run(["gcc", "-std=c11", *SAN, "-c", ORACLE_C, "-o", obj], check=True, capture_output=True, text=True)
    subprocess.run(["g++", "-std=c++17", *SAN, "-Wall", "-Wno-unused-function", "-I", SIM, "-I",
                    os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(CSRC, "api.cpp"),
                    os.path.join(CSRC, "partition.cpp"), os.path.join(SIM, "fake_device.cpp"),
                    os.path.join(SIM, "partition_sanitize.cpp"), obj, "-o", exe, "-lm"],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
