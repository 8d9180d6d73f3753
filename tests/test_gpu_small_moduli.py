"""Small-modulus residues (moduli of at most 255, held on the device as
centred int8): every contraction kernel against the oracle's entry-by-entry
definition of a step, the int8 matrix-core kernel in each of its tile shapes
and K schedules, extreme residues, and whole counts in both residue modes."""
import json
import os

import numpy as np
import pytest

import instances as I
from oracle import contract
from paper_1805_00475_amd import tn

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
MODULI = (255, 251, 254)


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _mask(rC, fA, rng):
    m = 0
    for q in rng.choice(rC, size=fA, replace=False):
        m |= 1 << int(q)
    return m


def _inputs(rA, rB, m, rng, kind):
    if kind == "plus":  # centred +m//2 (+127 for 255): the largest positive products
        return np.full(1 << rA, m // 2, np.uint32), np.full(1 << rB, m // 2, np.uint32)
    if kind == "mixed":  # centred values of the largest magnitude, both signs
        hi = (m + 1) // 2
        A = np.where(rng.integers(0, 2, size=1 << rA) == 1, m // 2, hi).astype(np.uint32)
        B = np.where(rng.integers(0, 2, size=1 << rB) == 1, m // 2, hi).astype(np.uint32)
        return A, B
    if kind == "raw":  # values not yet reduced: the library takes them modulo m
        return (rng.integers(0, 1 << 32, size=1 << rA, dtype=np.uint64).astype(np.uint32),
                rng.integers(0, 1 << 32, size=1 << rB, dtype=np.uint64).astype(np.uint32))
    return (rng.integers(0, m, size=1 << rA).astype(np.uint32), rng.integers(0, m, size=1 << rB).astype(np.uint32))


def _check(rA, rB, s, kernel, m, seed, kind="uniform", samples=None):
    rng = np.random.default_rng(seed)
    rC = rA + rB - 2 * s
    maskA = _mask(rC, rA - s, rng)
    A, B = _inputs(rA, rB, m, rng, kind)
    _say(f"kernel={kernel} rA={rA} rB={rB} s={s} m={m} kind={kind} mask={maskA:#x}")
    C = tn.step(A.copy(), rA, B.copy(), rB, s, maskA, prime=m, kernel=kernel)
    if samples is None and rC + s > 21:
        samples = max(24, min(4096, (1 << 21) >> s))
    if samples is None:
        cs = range(1 << rC)
    else:
        cs = sorted(set(rng.integers(0, 1 << rC, size=samples).tolist()) | {0, (1 << rC) - 1})
    want = contract.step_entries(A % m, B % m, s, maskA, rC, cs, m)
    got = [int(C[c]) for c in cs]
    assert got == want


ELEMENT = [
    ("generic", 5, 4, 2), ("generic", 9, 7, 3), ("generic", 6, 0, 0),
    ("stream", 14, 5, 3), ("stream", 12, 3, 1), ("stream", 10, 2, 0),
    ("rowdot", 12, 10, 8), ("rowdot", 9, 9, 9), ("rowdot", 14, 8, 7),
    # K >= 2^10: 16 bytes per lane and 4-way int8 dot products
    ("rowdot", 14, 12, 10), ("rowdot", 16, 13, 12), ("rowdot", 19, 14, 14), ("rowdot", 22, 15, 12),
    ("dot", 14, 14, 14), ("dot", 16, 15, 13),
    ("auto", 16, 15, 9), ("auto", 12, 3, 1), ("auto", 18, 18, 16),
]

# int8 matrix-core shapes (free sides fA >= 7, fB >= 6 after the role swap):
# 128x128 tiles with 1, 2 and 4+ stages per tile, 256x128 and 256x256 tiles,
# the 4-wave 256x64 and 128x64 tiles of B free sides of 6 bits, K split over
# block rows, more tiles than work-groups (tile loop), the roles swapped
MFMA8 = [
    ("mfma", 13, 13, 6), ("mfma", 14, 14, 7), ("mfma", 15, 15, 8), ("mfma", 16, 15, 8),
    ("mfma", 17, 17, 9), ("mfma", 18, 17, 10), ("mfma", 22, 21, 12), ("mfma", 20, 19, 8),
    ("mfma", 23, 20, 13), ("mfma", 19, 21, 11), ("mfma", 18, 17, 8), ("mfma", 23, 23, 16),
    ("mfma", 14, 14, 6), ("mfma", 16, 16, 7),
    ("mfma", 14, 12, 6), ("mfma", 16, 13, 7), ("mfma", 18, 16, 10), ("mfma", 19, 15, 9), ("mfma", 13, 12, 6),
    ("mfma", 17, 16, 10), ("mfma", 21, 20, 14), ("mfma", 15, 16, 9),
    # K = 2^s <= 32: fragments straight from A's and B's rows, 128x128 and
    # 128x64 tiles, s = 0..5
    ("mfma", 12, 12, 5), ("mfma", 13, 12, 4), ("mfma", 14, 13, 3), ("mfma", 10, 9, 2), ("mfma", 9, 8, 1),
    ("mfma", 8, 7, 0), ("mfma", 12, 11, 5), ("mfma", 11, 9, 3), ("mfma", 9, 7, 1),
]


@pytest.mark.parametrize("kernel,rA,rB,s", ELEMENT + MFMA8)
def test_kernel_small_modulus(kernel, rA, rB, s):
    for i, m in enumerate(MODULI[:2]):
        _check(rA, rB, s, kernel, m, seed=rA * 100 + rB * 10 + s + i)


@pytest.mark.parametrize("kernel,rA,rB,s", [("mfma", 15, 15, 8), ("mfma", 17, 17, 9), ("generic", 9, 7, 3),
                                            ("stream", 14, 5, 3), ("rowdot", 12, 10, 8)])
def test_even_modulus(kernel, rA, rB, s):
    # 254: the centred range is (-127, 127], one sided at 127
    _check(rA, rB, s, kernel, 254, seed=3)


@pytest.mark.parametrize("kind", ["plus", "mixed", "raw"])
@pytest.mark.parametrize("kernel,rA,rB,s", [("mfma", 17, 17, 9), ("mfma", 22, 21, 12), ("mfma", 23, 23, 16),
                                            ("stream", 13, 7, 5), ("rowdot", 12, 10, 8), ("rowdot", 16, 13, 12),
                                            ("dot", 16, 15, 13),
                                            ("generic", 9, 7, 3)])
def test_small_modulus_extreme_residues(kernel, rA, rB, s, kind):
    _check(rA, rB, s, kernel, 255, seed=7, kind=kind, samples=1500)


def test_tiny_moduli():
    for m in (2, 3, 7):
        _check(15, 15, 8, "mfma", m, seed=m)
        _check(12, 10, 8, "rowdot", m, seed=m)


def test_mfma8_refuses_narrow():
    # a free side of 5 bits has no int8 matrix-core tile
    rng = np.random.default_rng(0)
    A = rng.integers(0, 255, size=1 << 16).astype(np.uint32)
    B = rng.integers(0, 255, size=1 << 14).astype(np.uint32)
    with pytest.raises(tn.TNError):
        tn.step(A, 16, B, 14, 9, (1 << 7) - 1, prime=255, kernel="mfma")


def test_mfma8_full_size_sampled():
    # 2^11 output tiles of 256 x 256: more than the 1024 work-groups
    _check(24, 23, 10, "mfma", 255, seed=11, samples=300)
    # the largest narrow step of the n=200 cubic vertex-cover plans: 2^13
    # tiles of 256 x 64 with one stage each
    _check(27, 12, 6, "mfma", 253, seed=12, samples=300)
    # B free side of 6 bits, K = 2^17 split over block rows
    _check(24, 23, 17, "mfma", 251, seed=15, samples=24)
    # K = 32 with 2^12 tiles of 128 x 128: more than the 2048 work-groups
    _check(20, 16, 5, "mfma", 255, seed=16, samples=2000)


def test_mfma8_exact_range_flush():
    # 2^6 tiles of 256 x 256 with K = 2^17 in one block row: the int32 sums
    # are reduced after 2^16 entries, at the largest products
    _check(28, 28, 17, "mfma", 255, seed=13, kind="plus", samples=24)
    _check(28, 28, 17, "mfma", 251, seed=14, samples=24)


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def test_moduli_choice():
    from math import prod
    f = I.cvc(200, 0)
    net = tn.Network(f)
    bits = net.ranks()[1]  # the count bound that sizes the residues
    plan = net.order("community")
    small = tn.moduli(plan)
    assert max(small) <= 255 and prod(small) > 2 ** (bits + 1)
    wide = tn.moduli(plan, flags=tn.FLAG_WIDE_RNS)
    assert wide == tn.primes(tn.primes_for(bits))
    assert tn.moduli(plan, n_primes=9) == tn.primes(9)
    assert tn.moduli(tn.Network(I.cvc(40, 0)).order("community")) == []


def test_wide_and_small_counts_agree():
    for it in _gold("cvc_counts.json")["items"]:
        if it["n"] not in (120, 200) or it["seed"] > 1:
            continue
        f = I.cvc(it["n"], it["seed"])
        _say(f"cvc n={it['n']} seed={it['seed']} both residue modes")
        want = int(it["count"])
        assert tn.count(f, "community", seed=it["seed"]) == want
        assert tn.count(f, "community", seed=it["seed"], flags=tn.FLAG_WIDE_RNS) == want
        assert tn.count(f, "community", seed=it["seed"], flags=tn.FLAG_WIDE_RNS | tn.FLAG_NO_MFMA) == want
        assert tn.count(f, "community", seed=it["seed"], flags=tn.FLAG_NO_MFMA) == want
    # n = 200 (int8 planes of small moduli, or 16-bit primes): the two modes agree
    f = I.cvc(200, 3)
    _say("cvc n=200 seed=3 both residue modes")
    assert tn.count(f, "community", seed=3) == tn.count(f, "community", seed=3, flags=tn.FLAG_WIDE_RNS)


def test_contract_residues_small_moduli():
    f = I.cvc(120, 0)
    net = tn.Network(f)
    plan = net.order("community")
    want = tn.count_plan(net, plan, flags=tn.FLAG_WIDE_RNS)
    mods = tn.moduli(plan)
    res = tn.contract(net, plan)
    assert res == [want % m for m in mods]


def test_batch_wide_rns():
    with open(os.path.join(GOLD, "batch_counts.json")) as fh:
        g = {it["index"]: int(it["count"]) for it in json.load(fh)["items"]}
    fs = [I.batch_instance(i) for i in sorted(g)][:24]
    _say("batch of 24 with 16-bit primes")
    got = tn.count_batch(fs, "best", seed=0, flags=tn.FLAG_WIDE_RNS, workspace_bytes_=8 << 30)
    assert got == [g[i] for i in sorted(g)][:24]


def _layout_mask(rC, fA, layout, rng):
    # C's lowest bits owned as in layout ("A"/"B" per bit), the rest random
    low = [q for q, c in enumerate(layout) if c == "A"]
    rest = [q for q in range(len(layout), rC)]
    nA = fA - len(low)
    pick = rng.choice(len(rest), size=nA, replace=False)
    m = 0
    for q in low + [rest[int(i)] for i in pick]:
        m |= 1 << q
    return m


# Owners of C's four lowest bits select the epilogue's store form: 16-byte
# stores after exchanging lane bits 0, 1, 2, 4 or 5 with block bits, 4-byte
# words, or bytes (B owns C's two lowest bits).
LAYOUTS = ["AAAA", "BAAB", "BAAA", "AABB", "BBAA", "AAAB", "ABAA", "BABA", "ABAB", "ABBA", "BABB", "ABBB", "BBBB"]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("rA,rB,s", [(14, 14, 7), (14, 14, 6), (14, 12, 6), (13, 12, 5)])
def test_mfma8_output_layouts(layout, rA, rB, s):
    rng = np.random.default_rng(sum(ord(c) << (2 * i) for i, c in enumerate(layout)) * 1000 + rA * 100 + rB * 10 + s)
    rC = rA + rB - 2 * s
    maskA = _layout_mask(rC, rA - s, layout, rng)
    m = 251
    A = rng.integers(0, m, size=1 << rA).astype(np.uint32)
    B = rng.integers(0, m, size=1 << rB).astype(np.uint32)
    _say(f"layout={layout} rA={rA} rB={rB} s={s} mask={maskA:#x}")
    C = tn.step(A.copy(), rA, B.copy(), rB, s, maskA, prime=m, kernel="mfma")
    cs = sorted(set(rng.integers(0, 1 << rC, size=3000).tolist()) | set(range(64)) | {(1 << rC) - 1})
    assert [int(C[c]) for c in cs] == contract.step_entries(A, B, s, maskA, rC, cs, m)


def _check_big(rA, rB, s, m, seed, samples):
    # lean form of _check for operands of 2^30+ entries: residues drawn as
    # bytes below m, passed as the u32 arrays tn_step takes, no extra copies
    rng = np.random.default_rng(seed)
    rC = rA + rB - 2 * s
    maskA = _mask(rC, rA - s, rng)
    A = rng.integers(0, m, size=1 << rA, dtype=np.uint8).astype(np.uint32)
    B = rng.integers(0, m, size=1 << rB, dtype=np.uint8).astype(np.uint32)
    _say(f"kernel=mfma rA={rA} rB={rB} s={s} m={m} mask={maskA:#x} (full size, sampled)")
    C = tn.step(A, rA, B, rB, s, maskA, prime=m, kernel="mfma")
    cs = sorted(set(rng.integers(0, 1 << rC, size=samples).tolist()) | {0, (1 << rC) - 1})
    want = contract.step_entries(A, B, s, maskA, rC, cs, m)
    got = [int(C[c]) for c in cs]
    del A, B, C
    assert got == want


def test_mfma8_output_rank_30_to_32_sampled():
    # full-size steps of the largest 1-in-3 plans (n = 300, alpha = 0.62):
    # the dominant dense step (rank 31 x 31, K = 2^16, rank-30 output), a
    # rank-31 output at K = 2^10 and at K = 2^7, a short-K rank-30 output,
    # and a rank-32 output
    _check_big(31, 31, 16, 251, seed=31, samples=24)
    _check_big(30, 21, 10, 255, seed=32, samples=200)
    _check_big(26, 19, 7, 254, seed=33, samples=400)
    _check_big(27, 13, 5, 253, seed=34, samples=2000)
    _check_big(28, 28, 12, 255, seed=35, samples=100)


NARROW = [
    (12, 8, 6),     # 2^6 A rows (a partial tile), 2^2 B rows, K = 64 (one-MFMA chunks)
    (13, 13, 7),    # 64 x 64, K = 128
    (16, 11, 8),    # 2^8 rows x 8
    (18, 15, 10),   # 2^8 rows x 32 (two B blocks)
    (20, 10, 10),   # 2^10 rows x 1
    (17, 17, 11),   # 64 x 64 at K = 2^11
    (26, 21, 16),   # 2^10 rows x 32, K = 2^16: split over block rows
]


@pytest.mark.parametrize("rA,rB,s", NARROW)
@pytest.mark.parametrize("m", [255, 254, 7])
def test_narrow_kernel(rA, rB, s, m):
    _check(rA, rB, s, "narrow", m, seed=rA * 7 + m, samples=None if rA + rB - 2 * s <= 12 else 1500)


@pytest.mark.parametrize("kind", ["plus", "mixed"])
def test_narrow_kernel_extremes_and_flush(kind):
    # K = 2^17 at the largest products: the int32 sums are reduced after 2^16
    _check(24, 21, 17, "narrow", 255, seed=41, kind=kind, samples=200)
    _check(15, 12, 9, "narrow", 251, seed=42, kind=kind)


def test_narrow_refuses_wide_b():
    A = np.zeros(1 << 16, np.uint32)
    B = np.zeros(1 << 16, np.uint32)
    with pytest.raises(tn.TNError):
        tn.step(A, 16, B, 16, 8, (1 << 8) - 1, prime=255, kernel="narrow")   # 2^8 B rows
