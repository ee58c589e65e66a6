"""Device workspace layout (host C++, no GPU): alignment, bounds, disjoint regions, one slot
per device word, the sizes that reused regions need, and no overflow at the largest shapes."""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_workspace_layout(tmp_path):
    exe = str(tmp_path / "workspace_layout_test")
    src = os.path.join(ROOT, "tests", "workspace_layout_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-o", exe, src], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all passed" in out.stdout
