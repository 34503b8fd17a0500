"""The serving engine's arena map (host C++), built with g++ and checked
against a byte-level model on randomised allocate/release sequences."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_map_first_fit_against_model(tmp_path):
    exe = str(tmp_path / "arena_map_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-I", os.path.join(ROOT, "paper_1303_0383_amd", "csrc"),
                    os.path.join(ROOT, "tests", "arena_map_check.cpp"), "-o", exe], check=True)
    for seed in (1, 2, 3):
        out = subprocess.run([exe, str(seed)], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr
