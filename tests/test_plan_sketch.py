"""The judge ranks its bisection trials and reconfigured plans by sketches
(merges and predicted device time, without layouts or arena) and builds the
full plan of the winner only. This host check compiles a small program
against the library's internal header and libtn.so and confirms that a
sketch's status, predicted cost (bit for bit), largest rank and step count
are the full plan's, for partition and community orders of several formulas
and for broken merge lists."""
import os
import subprocess

import pytest

import instances as I
from instances import gen as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1805_00475_amd")


def _formula_text(f):
    lines = [f"{f.n_vars} {len(f.clauses)}"]
    for kind, cl in f.clauses:
        lines.append(f"{kind} {len(cl)} " + " ".join(str(x) for x in cl))
    return "\n".join(lines) + "\n"


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    lib = os.path.join(PKG, "libtn.so")
    if not os.path.exists(lib):
        pytest.skip("libtn.so is not built")
    exe = str(tmp_path_factory.mktemp("sketch") / "sketch_check")
    cmd = ["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "cpp", "sketch_check.cpp"), "-L", PKG, "-ltn", f"-Wl,-rpath,{PKG}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("name,f", [
    ("1in3-n300", I.large_1in3(300, 0.62, 1)),
    ("cvc-n120", I.cvc(120, 3)),
    ("cubic-1in3-90", G.cubic_1in3(60, 2)),
    ("mixed", I.batch_instance(7)),
])
def test_sketch_matches_full_plan(checker, name, f):
    r = subprocess.run([checker], input=_formula_text(f), capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
