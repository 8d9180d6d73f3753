"""O-A: brute-force enumeration of satisfying assignments.

The count of a formula F over n boolean variables is
    #F = sum over x in {0,1}^n of prod over clauses c of sat_c(x)
(the partition function of Eq. 2 in the zero-temperature limit, Sec. 2.1).
A literal +v is true when x_v = 1 and -v when x_v = 0 (negated indices,
Sec. 2.1). An OR clause is satisfied when at least one literal is true
(Eq. 3); an exactly-one clause when precisely one literal is true (Eq. 6);
a parity (XOR) clause when an odd number of literals is true (#XORSAT, one
of the other clause types Sec. 4 names). Literals are counted per occurrence.
An empty OR clause is therefore never satisfied, and an empty exactly-one or
parity clause neither (zero literals are true, not one, and zero is even).

Variable v (1-based) is bit v-1 of the assignment index x.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
OR = 0
EXACTLY_ONE = 1
XOR = 2


def clause_true_count(x: np.ndarray, lits) -> np.ndarray:
    """Number of true literals of one clause for every assignment in ``x``."""
    cnt = np.zeros(x.shape, dtype=np.int64)
    for lit in lits:
        bit = (x >> np.uint64(abs(lit) - 1)) & np.uint64(1)
        if lit < 0:
            bit = np.uint64(1) - bit
        cnt += bit.astype(np.int64)
    return cnt


def count_numpy(formula, chunk_bits: int = 20) -> int:
    """Enumerate all 2^n assignments with numpy (practical for n <= ~26)."""
    n = formula.n_vars
    total = 0
    chunk = 1 << min(n, chunk_bits)
    for start in range(0, 1 << n, chunk):
        x = np.arange(start, start + chunk, dtype=np.uint64)
        ok = np.ones(chunk, dtype=bool)
        for kind, lits in formula.clauses:
            t = clause_true_count(x, lits)
            if kind == OR:
                ok &= t >= 1
            elif kind == EXACTLY_ONE:
                ok &= t == 1
            elif kind == XOR:
                ok &= (t & 1) == 1
            else:
                raise ValueError(f"unknown clause kind {kind}")
        total += int(ok.sum())
    return total


_lib = None


def _load_c():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "libbruteforce.so")
        if not os.path.exists(path):
            build_c()
        _lib = ctypes.CDLL(path)
        _lib.bf_count.restype = ctypes.c_int
        _lib.bf_count.argtypes = [
            ctypes.c_int, ctypes.c_int,
            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
            ctypes.POINTER(ctypes.c_uint8), ctypes.c_int,
            ctypes.POINTER(ctypes.c_uint64)]
    return _lib


def build_c() -> str:
    """Compile ``bruteforce.c`` into ``libbruteforce.so`` next to it."""
    src = os.path.join(_HERE, "bruteforce.c")
    out = os.path.join(_HERE, "libbruteforce.so")
    import subprocess
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", out + ".tmp", src])
    os.replace(out + ".tmp", out)
    return out


def count_c(formula, threads: int = 0) -> int:
    """Same enumeration in plain C with OpenMP over the assignment range."""
    if formula.n_vars > 40:
        raise ValueError("brute force is limited to n <= 40")
    lib = _load_c()
    ptr, lits, kinds = formula.arrays()
    P = (ctypes.c_int32 * len(ptr))(*ptr)
    L = (ctypes.c_int32 * max(1, len(lits)))(*lits)
    K = (ctypes.c_uint8 * max(1, len(kinds)))(*kinds)
    out = ctypes.c_uint64(0)
    rc = lib.bf_count(formula.n_vars, formula.n_clauses, P, L, K, threads, ctypes.byref(out))
    if rc != 0:
        raise ValueError(f"bf_count failed with {rc}")
    return int(out.value)


def count(formula) -> int:
    """Brute-force count, picking numpy or C by size."""
    if formula.n_vars <= 18:
        return count_numpy(formula)
    return count_c(formula)
