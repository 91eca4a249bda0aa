"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (g++,
host code only).  One driver sweeps the planner and the modular-path
parameter code over shapes, dtypes, degenerate devices and forced tiles /
splits and checks every plan's invariants (tiles from the menu, splits
covering k exactly once, Theorem 1, workspace), grid fitting, and the CRT
constants (T_l = 1 mod p_l, 0 mod the others).  A second one checks the
planner's L2 <-> memory traffic model against a walk over every work item."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1908_09606_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "planner_sweep")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "host", "planner_sweep.cpp"),
           os.path.join(CSRC, "planner.cpp"), os.path.join(CSRC, "crt.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "planner sweep ok" in r.stdout
    assert "runtime error" not in r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_q_ea_model_equals_item_walk_under_asan_ubsan(tmp_path):
    """The planner's traffic model counts each wave's distinct panels from the
    raster's structure; a driver compares it, bit for bit, with a walk over
    every work item of 20000 random launches (ragged sizes, splits, raster
    groups taller than the matrix, 1..8 XCDs, 1..130 slots per XCD)."""
    exe = str(tmp_path / "q_ea_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "host", "q_ea_check.cpp"),
           os.path.join(CSRC, "planner.cpp"), os.path.join(CSRC, "crt.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "q_ea check ok" in r.stdout
