"""The clustering builder's merge-partner rule, run on the host (g++) with the kernel's own header:
every round of the build must merge at least one pair, also on inputs full of exact ties."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_clustering_round_merges(tmp_path):
    exe = tmp_path / "ploc_rounds"
    src = os.path.join(ROOT, "tests", "ploc_rounds.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK corners_of_a_box" in r.stdout
