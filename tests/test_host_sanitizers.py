"""The library's host runtime (runtime.cpp, mesh_step.cpp: validation,
request staging, the work-queue and job builders, the autotuner and its
cache, the continuous-batching scheduler) built with g++ against a CPU
stand-in of the HIP runtime (tests/host_harness) and run under
AddressSanitizer + UndefinedBehaviorSanitizer and under ThreadSanitizer.
No GPU is involved: the kernel launchers are stubs.

Scenarios: every entry point and its argument errors; every device
allocation of a client's sequence made to fail in turn (E_NOMEM or E_DEVICE,
no device block leaked) and host allocations failing by std::bad_alloc
(E_NOMEM, no exception across the C-ABI, no leaked in-flight count); six
client threads submitting, polling, waiting and cancelling on one context
while another reads its statistics (no data race)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "host_harness")
SOURCES = [os.path.join(ROOT, "paper_1504_00084_amd", "csrc", "runtime.cpp"),
           os.path.join(ROOT, "paper_1504_00084_amd", "csrc", "mesh_step.cpp"),
           os.path.join(HARNESS, "stub_kernels.cpp"), os.path.join(HARNESS, "harness.cpp")]
INCLUDES = ["-I" + HARNESS, "-I" + os.path.join(ROOT, "include"),
            "-I" + os.path.join(ROOT, "paper_1504_00084_amd", "csrc")]


def build(tmp, name, sanitize, defines=()):
    exe = os.path.join(tmp, name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + sanitize] + INCLUDES + \
        ["-D" + d for d in defines] + SOURCES + ["-o", exe, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    return exe


def run(exe, scenario, tmp):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    res = subprocess.run([exe, scenario, str(tmp)], capture_output=True, text=True, timeout=600, env=env)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert "WARNING: ThreadSanitizer" not in out, out[-4000:]
    return out


@pytest.fixture(scope="module")
def asan(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    return build(str(tmp_path_factory.mktemp("asan")), "harness_asan", "address,undefined")


@pytest.mark.parametrize("scenario", ["abi", "nomem", "threads"])
def test_host_runtime_under_asan_ubsan(asan, scenario, tmp_path):
    out = run(asan, scenario, tmp_path)
    assert "all checks passed" in out


def test_batch_split_into_launches_under_asan(tmp_path):
    """A build whose launch item limit is 3000 instead of 2^32 - 2^20: a
    batch of four requests of 1160 items each runs in two FP32 launches
    (every request OK), and a request of 3016 items is refused."""
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = build(str(tmp_path), "harness_split", "address,undefined", ["MESH_SDD_MAX_LAUNCH_ITEMS=3000u"])
    out = run(exe, "split", tmp_path)
    assert "all checks passed" in out


def test_scheduler_under_tsan(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = build(str(tmp_path), "harness_tsan", "thread")
    out = run(exe, "threads", tmp_path)
    assert "all checks passed" in out
