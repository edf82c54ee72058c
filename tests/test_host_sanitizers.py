"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (gcc/g++,
CPU only, no GPU code):

- the library's host setup (csrc/setup.cpp: lattice, local pair lists and
  groups, reciprocal vectors, overlap, Boys table) on a skewed cell with s, p
  and d shells and on invalid inputs (tests/host/setup_sanitized.cpp);
- the CPU oracle's C loops (oracle/oracle.c) on a skewed cell with s, p and
  spherical d shells (tests/host/oracle_sanitized.c)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_22278_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_setup_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "setup_sanitized")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__host__=", "-D__device__=", f"-I{CSRC}",
           os.path.join(ROOT, "tests", "host", "setup_sanitized.cpp"), os.path.join(CSRC, "setup.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.count("ok:") == 2 and r.stdout.count("rejected as expected") == 3


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", f"-I{os.path.join(ROOT, 'oracle')}",
           os.path.join(ROOT, "tests", "host", "oracle_sanitized.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert "bad 0" in r.stdout
