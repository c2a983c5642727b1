"""Host-only checks that the product path stays separate from the oracle and
fails loudly without its HIP library."""
import ast
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2201_00451_amd")


def imported_modules(path):
    tree = ast.parse(open(path).read())
    mods = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            mods.update(a.name for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.module:
            mods.add(node.module)
    return mods


def test_package_never_imports_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith(".py"):
                mods = imported_modules(os.path.join(dirpath, f))
                assert not any(m.split(".")[0] == "oracle" for m in mods), f


def test_hip_sources_do_not_reference_the_oracle():
    for dirpath, _, files in os.walk(os.path.join(PKG, "csrc")):
        for f in files:
            assert "oracle" not in open(os.path.join(dirpath, f)).read().lower(), f


def test_missing_library_raises(tmp_path):
    from paper_2201_00451_amd import binding
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2201_00451_amd import binding\n"
            "try:\n"
            "    binding.load_library(%r)\n"
            "except binding.FstatError as e:\n"
            "    print('raised', e.status)\n") % (ROOT, str(tmp_path / "missing.so"))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, check=True)
    assert out.stdout.strip() == f"raised {binding.FSTAT_EUNSUPPORTED}"


def test_bench_refuses_several_gpus():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
