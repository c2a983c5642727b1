"""Host-only checks of library internals compiled from the same sources
(no GPU is used): the per-template prologue's analytic sky derivatives."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_prologue_sky_derivatives(tmp_path):
    exe = tmp_path / "prologue_derivatives"
    subprocess.run(["/opt/rocm/bin/hipcc", "-std=c++17", "-O1",
                    "-I", os.path.join(ROOT, "paper_2201_00451_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host", "prologue_derivatives.cpp"),
                    "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout
