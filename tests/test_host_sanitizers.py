"""The library's host-only code under AddressSanitizer and UBSan (CPU only).

The real Schur decomposition used by the Schur-basis seed (schur_host.cpp) is
plain C++: it is compiled with g++ together with a small driver
(tests/host/schur_driver.cpp) under -fsanitize=address,undefined and run on
random, rotation-block and defective matrices of several sizes, including
n = 1, 2, 3.  Any out-of-bounds access, leak or undefined behaviour aborts the
run; the driver also checks A = Z T Z^T and the orthogonality of Z.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_real_schur_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "schur_driver")
    src = [os.path.join(ROOT, "tests", "host", "schur_driver.cpp"),
           os.path.join(ROOT, "paper_2312_08201_amd", "csrc", "schur_host.cpp")]
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", exe] + src
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    # verify_asan_link_order=0: the environment may preload other libraries
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ALL OK" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_streamk_partition_under_asan_and_ubsan(tmp_path):
    """The stream-K partition of the GEMM launches (streamk.h): exact coverage
    of every (tile, K-tile) iteration, one write per (tile, segment), segment
    counts that match the consumer's, writes inside the reserved partial rows,
    and a permutation for the XCD-aware range order, over active row counts
    1..M, grids 1..1024 and K-tile counts 1..512."""
    exe = str(tmp_path / "streamk_check")
    src = [os.path.join(ROOT, "tests", "host", "streamk_check.cpp")]
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", exe] + src
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ALL OK" in r.stdout
