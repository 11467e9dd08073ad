"""Host-side checks of the batched plan code (plan build, graph parameter
updates, eviction, adjoint launches) on the CPU.

``batched_abi.hip``, ``host_checks.hip`` and ``tune_table.hip`` are compiled for the host only
and linked, with AddressSanitizer and UndefinedBehaviorSanitizer, against a
CPU stand-in of the HIP runtime (``tests/plan_host/hip_stub.cpp``) whose
kernel table lists each kernel's parameters.  The stand-in reads every
kernel argument through the parameter arrays the plan code passes (so a
short or dangling array is an AddressSanitizer error), checks pointer
arguments against live allocations, and models launches in flight: freeing
memory, destroying a graph executable or rewriting its node parameters while
a launch of it may still run are reported as violations.
"""

from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1110_5450_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "plan_host")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]

pytestmark = pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang is not installed")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan_host")
    srcs = [os.path.join(CSRC, "batched_abi.hip"), os.path.join(CSRC, "host_checks.hip"),
            os.path.join(CSRC, "tune_table.hip"),
            os.path.join(HOST, "stub_kernels.cpp"), os.path.join(HOST, "hip_stub.cpp"),
            os.path.join(HOST, "plan_driver.cpp")]
    objs = []
    for s in srcs:
        o = str(d / (os.path.basename(s) + ".o"))
        cmd = [CLANG, "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g",
               "-fno-omit-frame-pointer", "-Wno-unused-value", "-Wno-unused-result", *SAN, "-I", os.path.join(ROOT, "include"), "-c", s, "-o", o]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr[-4000:]
        objs.append(o)
    exe = str(d / "plan_driver")
    cmd = [CLANG, *objs, "-fsanitize=address,undefined", "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr[-4000:]
    return exe


def _run(exe, mode):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe, mode], capture_output=True, text=True, timeout=300, env=env)


def test_stand_in_reports_planted_hazards(driver):
    r = _run(driver, "selftest")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "rewritten while a launch of the executable is in flight" in r.stdout
    assert "destroyed while a launch of it is in flight" in r.stdout
    assert "hipFree of memory that a launch in flight uses" in r.stdout


def test_plans_evictions_and_updates_are_clean(driver):
    r = _run(driver, "plans")
    print(r.stdout)
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stdout + r.stderr[-6000:]
    assert "violations 0" in r.stdout
    launches = int(re.search(r"graph launches (\d+)", r.stdout).group(1))
    updates = int(re.search(r"parameter updates (\d+)", r.stdout).group(1))
    assert launches == 3 * 42 and updates > 0


def test_batched_autotuner_records_and_rebuilds(driver):
    r = _run(driver, "tune")
    print(r.stdout)
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stdout + r.stderr[-6000:]
    assert "violations 0" in r.stdout
    m = re.search(r"tuned config (\d+) .* automatic config (\d+)", r.stdout)
    assert m and m.group(1) == m.group(2)


def _param_count(src: str, name: str) -> int:
    m = re.search(r"__global__[^;{]*?\b" + name + r"\s*\(", src)
    assert m, name
    i, depth = m.end(), 1
    j = i
    while depth:
        depth += {"(": 1, ")": -1}.get(src[j], 0)
        j += 1
    params = src[i:j - 1]
    depth, n = 0, 1
    for ch in params:
        if ch in "(<[":
            depth += 1
        elif ch in ")>]":
            depth -= 1
        elif ch == "," and depth == 0:
            n += 1
    return n


def test_stand_in_kernel_table_matches_the_kernel_sources(driver):
    r = _run(driver, "table")
    table = dict((ln.split()[0], int(ln.split()[1])) for ln in r.stdout.split("\n") if ln.strip())
    src = open(os.path.join(CSRC, "batched_kernels.hip")).read() + open(os.path.join(CSRC, "backward_kernels.hip")).read()
    for name, n in table.items():
        assert _param_count(src, name) == n, name
