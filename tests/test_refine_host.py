"""Host check of the local reconfiguration of contraction trees (the
judge's last stage): a small program compiled against the library's
internal header and libtn.so reconfigures partition orders of several
formulas to convergence and checks that each result is a valid plan, no
more costly under the cost model, no larger in its largest rank, and the
same when run again."""
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
    if not os.path.exists(os.path.join(PKG, "libtn.so")):
        pytest.skip("libtn.so is not built")
    exe = str(tmp_path_factory.mktemp("refine") / "refine_check")
    cmd = ["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "cpp", "refine_check.cpp"), "-L", PKG, "-ltn", f"-Wl,-rpath,{PKG}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("name,f", [
    ("1in3-n250", I.large_1in3(250, 0.66, 2)),
    ("cvc-n200", I.cvc(200, 1)),
    ("cubic-1in3-150", G.cubic_1in3(100, 3)),
])
def test_reconfiguration(checker, name, f):
    r = subprocess.run([checker], input=_formula_text(f), capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
