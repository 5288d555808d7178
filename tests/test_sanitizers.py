"""The CPU oracle and the library's host BVH builder and node compressor
under AddressSanitizer and UndefinedBehaviorSanitizer (gcc/g++; host code
only): seeded random scenes, every intersector, query and node layout of the
oracle, leaf sizes 1..7 of the builder (drivers in tests/sanitize/)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-ffp-contract=off"]


def _run(cmd_compile, exe, expect):
    r = subprocess.run(cmd_compile, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert p.returncode == 0, (p.returncode, p.stdout[-2000:], p.stderr[-4000:])
    assert expect in p.stdout
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c11", *FLAGS, "-pthread", os.path.join(HERE, "sanitize", "oracle_driver.c"),
          "-o", exe, "-lm"], exe, "oracle ok")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "builder_driver")
    _run(["g++", "-std=c++17", *FLAGS, os.path.join(HERE, "sanitize", "builder_driver.cpp"),
          "-o", exe], exe, "builder ok")
