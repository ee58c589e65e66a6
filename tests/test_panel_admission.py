"""Admission of the band reduction's panel kernels across streams (C++, no GPU): a model GPU in
which a panel kernel completes only once all its workgroups are resident never gets stuck
under the admission rule, while the two weaker rules it is compared with do."""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_panel_admission(tmp_path):
    exe = str(tmp_path / "panel_admission_test")
    src = os.path.join(ROOT, "tests", "panel_admission_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-o", exe, src], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all passed" in out.stdout
