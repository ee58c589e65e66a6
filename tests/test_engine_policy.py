"""Serving-engine scheduling policy (C++, no GPU) with a mock executor and a fake budget."""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_engine_policy(tmp_path):
    exe = str(tmp_path / "engine_policy_test")
    src = os.path.join(ROOT, "tests", "engine_policy_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-fsanitize=address,undefined",
                    "-o", exe, src], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all passed" in out.stdout
