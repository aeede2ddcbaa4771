"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU, no
device): the workspace allocator against a byte-level model of its region,
and the bin look-up tables and pair-bin volumes on random edge sets
(tests/host/heap_check.cpp, compiled here with the sanitizers on the host
pass only); and the device line transforms emulated on the CPU, one thread
per lane, under ThreadSanitizer and AddressSanitizer
(tests/host/fft_check.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "heap_check")
    cmd = [HIPCC, "-std=c++17", "-O1", "-g",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", ROOT, "-o", exe, os.path.join(HERE, "host", "heap_check.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host checks passed" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_line_transforms_on_the_cpu(tmp_path, sanitizer):
    """The device line transforms (csrc/pgx_fft.hpp, every two- and
    three-stage shape the kernels use) run on the CPU with one thread per lane
    and a barrier per exchange (tests/host/fft_check.cpp), against a direct
    DFT.  ThreadSanitizer shows that the exchanges are separated by the
    barriers; AddressSanitizer that no lane leaves its line."""
    exe = str(tmp_path / "fft_check")
    cmd = ["g++", "-std=c++20", "-O1", "-g", f"-fsanitize={sanitizer}", "-fno-sanitize-recover=all",
           "-I", os.path.join(HERE, "host", "emu"), "-o", exe, os.path.join(HERE, "host", "fft_check.cpp"),
           "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "line transform checks passed" in r.stdout
