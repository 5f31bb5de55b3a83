"""Host logic of the library on the CPU: the runtime, the block schedule and
the server, compiled against a stand-in HIP runtime whose kernel launchers
check every device range a kernel would touch (tests/host_emu).  The solver and
serving scenarios run under AddressSanitizer + UndefinedBehaviorSanitizer and,
where a ThreadSanitizer runtime is available, under ThreadSanitizer.

Regression cases: a status macro whose local shadowed the run's block size
(a null partial-residual buffer reached a kernel), and a finished request read
by the worker after the caller had deleted it.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_11673_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "host_emu")
SOURCES = [os.path.join(CSRC, f) for f in ("runtime.cpp", "schedule.cpp", "gram_plan.cpp")] + \
          [os.path.join(EMU, f) for f in ("emu_hip.cpp", "emu_kernels.cpp", "driver.cpp")]


def _build(tmpdir, compiler, flags, name):
    out = os.path.join(tmpdir, name)
    cmd = [compiler, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-include", "cstddef",
           "-I", EMU, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "c++", *SOURCES, "-o", out,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


@pytest.fixture(scope="module")
def asan_bin(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ is not available")
    return _build(str(tmp_path_factory.mktemp("emu")), "g++", ["-fsanitize=address,undefined"], "emu_asan")


def _run(binary, scenario, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([binary, scenario], capture_output=True, text=True, timeout=600, env=env)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.parametrize("scenario", ["solve", "sparse", "serve"])
def test_host_logic_in_bounds(asan_bin, scenario):
    rc, out = _run(asan_bin, scenario, {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "halt_on_error=1"})
    assert rc == 0 and "EMU OK" in out, out[-6000:]
    assert "EMU OOB" not in out and "runtime error" not in out, out[-6000:]


def test_server_has_no_data_races(tmp_path_factory):
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang):
        pytest.skip("no clang with a ThreadSanitizer runtime")
    binary = _build(str(tmp_path_factory.mktemp("emu_tsan")), clang, ["-fsanitize=thread"], "emu_tsan")
    rc, out = _run(binary, "serve", {"TSAN_OPTIONS": "halt_on_error=1"})
    assert rc == 0 and "EMU OK" in out and "ThreadSanitizer" not in out, out[-6000:]
