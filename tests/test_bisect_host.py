"""Host check of the partition order's balanced bisection: a small program
compiled against the library's internal graph header and libtn.so runs
``bisect`` on 3000 random weighted graphs of 2 to 24 vertices. Up to 12
vertices, where every split is tried, the cut must equal the lightest
balanced split found by brute force; above, the split must lie within the
balance window; always, the reported cut must be the split's."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1805_00475_amd")


def test_bisect_against_brute_force(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libtn.so")):
        pytest.skip("libtn.so is not built")
    exe = str(tmp_path / "bisect_check")
    cmd = ["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "cpp", "bisect_check.cpp"), "-L", PKG, "-ltn", f"-Wl,-rpath,{PKG}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:]
