"""The request server's HBM admission arena (csrc/arena.hpp, plain C++ with
no device calls), driven on the CPU under AddressSanitizer and
UndefinedBehaviorSanitizer: a long seeded sequence of first-fit allocations
and releases, checked after every step against a list of live blocks."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2001_02765_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_under_sanitizers(tmp_path):
    exe = str(tmp_path / "arena_driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I" + CSRC,
                    os.path.join(ROOT, "tests", "arena_driver.cpp"), "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    for seed in (1, 2, 3):
        r = subprocess.run([exe, str(seed)], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.startswith("ok")
