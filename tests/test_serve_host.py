"""The request server's host logic (admission, table cache, output arena,
round scheduling, completion) compiled with g++ against a fake device and
run over randomised workloads under the host address and undefined-behaviour
sanitizers: every request completes once, every edge is generated once, with
its own table, and the arena drains."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM = os.path.join(ROOT, "tests", "hostsim")
CSRC = os.path.join(ROOT, "paper_1905_03525_amd", "csrc")


@pytest.fixture(scope="module")
def sim_binary(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("hostsim") / "serve_sim")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-Wall", "-Wno-unused-function", "-I", SIM, "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "serve.cpp"),
           os.path.join(SIM, "fake_device.cpp"), os.path.join(SIM, "serve_sim.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_server_host_logic_randomised(sim_binary, seed):
    r = subprocess.run([sim_binary, "150", str(seed)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0"))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 errors" in r.stdout
