"""Host logic of the rank variant's search buckets, compiled on the CPU with the host
compiler and checked against brute force (tests/cpp/rank_buckets_check.cpp): monotone
bucket maps, exact bucket starts, the fewest search steps that cover the fullest bucket,
and the caps and modes respected."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_rank_buckets_against_brute_force(tmp_path):
    exe = tmp_path / "rank_buckets_check"
    subprocess.run(["g++", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_1801_03644_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "rank_buckets_check.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad=0" in out.stdout
