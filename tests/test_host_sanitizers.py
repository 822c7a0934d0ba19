"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The work schedules of the batched and 4D launches (ecc_schedule.cpp) and the
contribution-table builders (ecc_tables.cpp) are plain host C++: they are
compiled with g++ -fsanitize=address,undefined together with a checker
(tests/host/sched_check.cpp) that drives them over random fields and checks
that every schedule covers each field's units exactly once, keeps every item
within what the packed LDS bins may take between drains, and keeps every
tile's staged levels within its LDS slots (what the kernels rely on to stay in
bounds).  The run must end cleanly, with no sanitizer report.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_11740_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_schedules_and_tables_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sched_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", CSRC,
           os.path.join(CSRC, "ecc_schedule.cpp"), os.path.join(CSRC, "ecc_tables.cpp"),
           os.path.join(ROOT, "tests", "host", "sched_check.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, "400"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "rounds OK" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_affine_level_estimates_under_sanitizers(tmp_path):
    """The margins of the affine level estimate (ecc_levels.cpp) against a
    float32 replay of the kernels' estimate and settle steps
    (tests/host/levels_check.cpp): values at, next to and between all
    thresholds of several grids land on their exact level in every form."""
    exe = str(tmp_path / "levels_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", CSRC,
           os.path.join(CSRC, "ecc_levels.cpp"), os.path.join(ROOT, "tests", "host", "levels_check.cpp"),
           "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "level estimates OK" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
