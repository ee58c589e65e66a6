"""Schedule of a group run above the fused kernel's size (C++, no GPU): random groups advanced
round by round end at their last step and observe exactly at the multiples of obs_every."""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_group_schedule(tmp_path):
    exe = str(tmp_path / "group_schedule_test")
    src = os.path.join(ROOT, "tests", "group_schedule_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-o", exe, src], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all passed" in out.stdout
