"""Host check of the count bounds that size the residue system, beyond the
oracle-pinned cases of test_count_bound.py: a small program compiled
against the library's internal header and libtn.so checks on 600 random
formulas (OR, exactly-one and parity clauses, negations and repeated
literals, 4 to 20 variables) that every bound, the library's two and the
same elimination with mini-buckets of 1 to 4 other variables (one sum and
maxima, or Hoelder norms; fewest-neighbour or least-fill order), is at
least log2 of the count found by enumeration."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1805_00475_amd")


def test_bounds_against_enumeration(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libtn.so")):
        pytest.skip("libtn.so is not built")
    exe = str(tmp_path / "bound_check")
    cmd = ["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "cpp", "bound_check.cpp"), "-L", PKG, "-ltn", f"-Wl,-rpath,{PKG}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:]
