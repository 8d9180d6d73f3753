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
