"""Kernel-level parity: every contraction kernel (generic, streaming,
row-dot, int8-limb MFMA) on seeded random residues against the oracle's
entry-by-entry definition of a step, at sizes spanning several tiles and at
full workload sizes on sampled outputs."""
import numpy as np
import pytest

from oracle import contract, rns
from paper_1805_00475_amd import tn

pytestmark = pytest.mark.gpu
P = rns.largest_primes_below(65280, 8)


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _mask(rC, fA, rng):
    pos = rng.choice(rC, size=fA, replace=False)
    m = 0
    for q in pos:
        m |= 1 << int(q)
    return m


def _inputs(rA, rB, p, rng, kind="uniform"):
    if p is None:
        A = rng.integers(0, 1 << 62, size=1 << rA, dtype=np.uint64)
        B = rng.integers(0, 1 << 62, size=1 << rB, dtype=np.uint64)
        return A, B
    if kind == "max":
        return np.full(1 << rA, p - 1, np.uint32), np.full(1 << rB, p - 1, np.uint32)
    if kind == "half":
        # values around p/2, where the centred digit form switches sign
        A = (p // 2 + rng.integers(-3, 4, size=1 << rA)).astype(np.uint32)
        B = (p // 2 + rng.integers(-3, 4, size=1 << rB)).astype(np.uint32)
        return A, B
    A = rng.integers(0, p, size=1 << rA, dtype=np.int64).astype(np.uint32)
    B = rng.integers(0, p, size=1 << rB, dtype=np.int64).astype(np.uint32)
    return A, B


def _budget(rC, s, samples):
    # keep the oracle's entry-by-entry work near 2^21 products
    if samples is None and (rC + s) <= 21:
        return None
    return min(samples or 4096, max(64, (1 << 21) >> s))


def _check(rA, rB, s, kernel, p, seed, kind="uniform", samples=None):
    rng = np.random.default_rng(seed)
    rC = rA + rB - 2 * s
    fA = rA - s
    maskA = _mask(rC, fA, rng)
    A, B = _inputs(rA, rB, p, rng, kind)
    _say(f"kernel={kernel} rA={rA} rB={rB} s={s} p={p} kind={kind} mask={maskA:#x}")
    C = tn.step(A.copy(), rA, B.copy(), rB, s, maskA, prime=p, kernel=kernel)
    samples = _budget(rC, s, samples)
    if samples is None:
        cs = range(1 << rC)
    else:
        cs = sorted(set(rng.integers(0, 1 << rC, size=samples).tolist()) | {0, (1 << rC) - 1})
    want = contract.step_entries(A, B, s, maskA, rC, cs, p)
    got = [int(C[c]) for c in cs]
    assert got == want


SMALL = [
    ("generic", 5, 4, 2), ("generic", 9, 7, 3), ("generic", 3, 3, 3), ("generic", 6, 0, 0),
    ("stream", 14, 5, 3), ("stream", 12, 3, 1), ("stream", 13, 7, 5), ("stream", 10, 2, 0),
    ("rowdot", 12, 10, 8), ("rowdot", 9, 9, 9), ("rowdot", 14, 8, 7),
    ("mfma", 13, 12, 6), ("mfma", 18, 17, 8), ("mfma", 16, 15, 9), ("mfma", 21, 20, 14), ("mfma", 15, 14, 7),
    ("mfma", 22, 21, 15), ("mfma", 23, 22, 14), ("mfma", 17, 16, 10), ("mfma", 23, 23, 16),
    ("dot", 14, 14, 14), ("dot", 16, 15, 13), ("dot", 12, 12, 10),
    ("auto", 16, 15, 9), ("auto", 12, 3, 1), ("auto", 18, 18, 16),
]


@pytest.mark.parametrize("kernel,rA,rB,s", SMALL)
def test_kernel_rns(kernel, rA, rB, s):
    for i, p in enumerate(P[:2]):
        _check(rA, rB, s, kernel, p, seed=rA * 100 + rB * 10 + s + i)


@pytest.mark.parametrize("kind", ["max", "half"])
@pytest.mark.parametrize("kernel,rA,rB,s", [("mfma", 16, 15, 9), ("mfma", 23, 22, 16), ("mfma", 23, 23, 16),
                                            ("stream", 13, 7, 5),
                                            ("rowdot", 12, 10, 8), ("generic", 9, 7, 3)])
def test_kernel_extreme_residues(kernel, rA, rB, s, kind):
    _check(rA, rB, s, kernel, P[-1], seed=7, kind=kind, samples=2000)


@pytest.mark.parametrize("kernel,rA,rB,s", [("generic", 9, 7, 3), ("stream", 14, 5, 3), ("rowdot", 12, 10, 8),
                                            ("dot", 16, 15, 13)])
def test_kernel_u64(kernel, rA, rB, s):
    _check(rA, rB, s, kernel, None, seed=5, samples=2000)


def test_mfma_refuses_small_or_u64():
    rng = np.random.default_rng(0)
    A, B = _inputs(10, 10, P[0], rng)
    with pytest.raises(tn.TNError):
        tn.step(A, 10, B, 10, 5, (1 << 5) - 1, prime=P[0], kernel="mfma")  # K = 32 < 64


@pytest.mark.parametrize("kernel,rA,rB,s", [("mfma", 24, 23, 10), ("stream", 28, 3, 1), ("stream", 27, 5, 2),
                                            ("dot", 22, 22, 22), ("mfma", 22, 24, 15)])
def test_kernel_full_size_sampled(kernel, rA, rB, s):
    # shapes of the largest steps of the n=200 cubic vertex-cover plans
    _check(rA, rB, s, kernel, P[3], seed=11, samples=400)


def test_mfma_exact_range_flush():
    # K = 2^16 over 64 output tiles of 128 x 128: no K split, so the exact
    # int32 sums are reduced once in the middle of K (after 2^15 entries)
    _check(26, 26, 16, "mfma", P[5], seed=13, samples=300)


def test_mfma_narrow_tile_wide_k():
    # 128 x 64 tiles (B's free side of 6 bits) with K = 2^17: the launch
    # splits K into exact ranges of at most 2^15 entries
    _check(24, 23, 17, "mfma", P[6], seed=17, samples=300)
