"""The count bound that sizes the residue system (block products, for
formulas of more than 63 variables): never below the true count. Formulas on
20-22 variables, padded with unused variables past 63 (each doubles the
count), are counted by the oracle's brute force; 2^count_bits must be at
least the count, for OR, exactly-one and parity clauses, negations, repeated
and complementary literals, long clauses and empty clauses."""
import pytest

import instances as I
from oracle import brute
from paper_1805_00475_amd import tn


def _padded(f, pad):
    return I.Formula(f.n_vars + pad, list(f.clauses), f.name)


def _check(f, pad=44):
    want = brute.count_c(f) << pad
    bits = tn.Network(_padded(f, pad)).ranks()[1]
    assert want <= 1 << bits, (want.bit_length(), bits)
    return bits


def test_bound_exactly_one():
    rng = I.Rng(71)
    for _ in range(12):
        f = I.exactly_one_3(21, rng.below(18), rng)
        _check(f)
    # denser: the bound must drop well below n
    f = I.exactly_one_3(22, 14, I.Rng(5))
    assert _check(f) < 22 + 44  # below 2^n (never below 64 bits: small moduli stay)


@pytest.mark.parametrize("k", [4, 5])
def test_bound_one_in_k_and_parity(k):
    rng = I.Rng(90 + k)
    for _ in range(6):
        _check(I.exactly_one_k(21, rng.below(10), k, rng))
        _check(I.xor_k(21, rng.below(16), k, rng))


def test_bound_mixed_negations_repeats():
    rng = I.Rng(404)
    for _ in range(24):
        f = I.random_mixed_formula(20, rng.below(30), rng, max_len=6)
        f.clauses = [(k if rng.below(3) else I.XOR, c) for k, c in f.clauses]
        _check(f)


def test_bound_empty_clause_and_cover():
    f = I.Formula(20, [(I.OR, [1, 2]), (I.EXACTLY_ONE, [])])
    assert brute.count_c(f) == 0
    _check(f)
    g = I.cvc(20, 0)
    _check(g)


def _check_large(f, pad):
    # at least 160 variables in all: blocks of up to 96, counted by
    # elimination (or split again when too wide); the oracle counts the core
    from oracle import elim
    assert f.n_vars + pad >= 160
    want = elim.count(f) << pad
    bits = tn.Network(_padded(f, pad)).ranks()[1]
    assert want <= 1 << bits, (want.bit_length(), bits)
    return bits


def test_bound_elimination_blocks():
    rng = I.Rng(2024)
    for _ in range(4):
        _check_large(I.exactly_one_3(40, 26, rng), 130)
    for _ in range(4):
        f = I.random_mixed_formula(34, 30, rng, max_len=4)
        f.clauses = [(k if rng.below(3) else I.XOR, c) for k, c in f.clauses]
        _check_large(f, 130)
    # the headline family at full size against the stored oracle counts
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c3_1in3_counts.json")))
    for it in gold["items"][:6]:
        f = I.large_1in3(it["n"], it["alpha"], it["seed"])
        bits = tn.Network(f).ranks()[1]
        assert int(it["count"]) <= 1 << bits and bits < it["n"]


def test_bound_wide_blocks_split_again():
    # dense parity systems of 90 variables: eliminating a block of them would
    # need tables far past the width cap, so blocks are split again; the GF(2)
    # rank formula counts them
    from oracle import closed
    rng = I.Rng(77)
    for m in (60, 80, 100):
        # a planted solution keeps the system satisfiable
        x = [rng.coin() for _ in range(90)]
        f = I.Formula(90)
        for _ in range(m):
            vs = []
            while len(vs) < 3:
                v = rng.below(90)
                if v not in vs:
                    vs.append(v)
            lits = [v + 1 for v in vs]
            if sum(x[v] for v in vs) % 2 == 0:
                lits[0] = -lits[0]
            f.clauses.append((I.XOR, lits))
        want = closed.xorsat_count(f) << 80
        assert want > 0
        bits = tn.Network(_padded(f, 80)).ranks()[1]
        assert want <= 1 << bits, (want.bit_length(), bits)
