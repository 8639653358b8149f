"""The eviction rule of the library's cached work-lists (blocked rotation):
least recently used, at most 8 unpinned entries, and entries used under
stream capture pinned for good (a captured graph keeps their device
pointers).  The rule lives in a host-only header; this test compiles a small
checker against it with the host compiler and runs it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pinned_lru_eviction_rule(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "pinned_lru_check"
    src = os.path.join(ROOT, "tests", "pinned_lru_check.cpp")
    inc = os.path.join(ROOT, "paper_0909_5662_amd", "csrc")
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-I", inc, src, "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0 and res.stdout.strip() == "ok", res.stdout + res.stderr
