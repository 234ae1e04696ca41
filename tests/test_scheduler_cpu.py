"""The request server's scheduling policy (arena allocator, admission,
anti-starvation, demand-sized groups, release of idle groups) on the host, with a fake executor.

tests/scheduler_driver.cpp includes the policy header the server is built
from and simulates groups whose chunks finish in one round; it is compiled
here with the host compiler (with address and undefined-behaviour checks)."""

import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
SCENARIOS = (["arena", "fifo_join", "busy_group", "starvation", "small_groups", "small_idle_groups",
              "serving"] + [f"serving_mix_{seed}" for seed in range(1, 21)])


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path_factory.mktemp("sched") / "scheduler_driver"
    cmd = [cxx, "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
           "-I", str(ROOT / "paper_1901_07294_amd" / "csrc"),
           str(ROOT / "tests" / "scheduler_driver.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def test_scheduler_policy_with_fake_executor(driver):
    out = subprocess.run([str(driver)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    for name in SCENARIOS:
        assert f"PASS {name}" in out.stdout, out.stdout
