"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each test patches one oracle function with a plausible bug -- a dropped
term, a wrong sign or index, an off-by-one in a clause rule -- and checks
that at least one pin that does not come from the oracle then fails.
"""
import numpy as np
import pytest

import instances as I
from oracle import brute, closed, contract, elim, rns, tensors


def _contract_pins_hold():
    """Pairwise contractor against pins fixed outside the contractor."""
    checks = [
        (I.vertex_cover_formula(I.prism_graph(5)), 81),
        (I.vertex_cover_formula(I.complete_graph(4)), 5),
        (I.perfect_matching_formula(I.prism_graph(4)), 9),
        (I.Formula(5, []), 32),
    ]
    for f, want in checks:
        if contract.count_exact(f) != want:
            return False
    rng = I.Rng(77)
    for _ in range(12):
        f = I.random_mixed_formula(6, 5, rng)
        if contract.count_exact(f) != brute.count(f):
            return False
    return True


def _rns_pins_hold():
    # 80 variables: intermediate entries exceed 2^31, so every residue is
    # full-width and each limb product matters
    f = I.vertex_cover_formula(I.prism_graph(40))
    return contract.count_rns(f, rns.largest_primes_below(1 << 31, 4)) == closed.prism_vertex_covers(40)


def test_unpatched_pins_hold():
    assert _contract_pins_hold()
    assert _rns_pins_hold()


def test_or_tensor_accepting_all_false(monkeypatch):
    orig = tensors.clause_tensor

    def bad(kind, negated):
        t = orig(kind, negated)
        if kind == tensors.OR and len(negated):
            t = t.copy()
            t[(0,) * len(negated)] = 1
        return t
    monkeypatch.setattr(tensors, "clause_tensor", bad)
    assert not _contract_pins_hold()


def test_exactly_one_off_by_one(monkeypatch):
    import itertools
    orig = tensors.clause_tensor

    def bad(kind, negated):
        if kind != tensors.EXACTLY_ONE:
            return orig(kind, negated)
        d = len(negated)
        t = np.zeros((2,) * d, dtype=object)
        for idx in itertools.product((0, 1), repeat=d):
            eff = [i ^ int(bool(n)) for i, n in zip(idx, negated)]
            t[idx] = 1 if sum(eff) <= 1 else 0
        return t
    monkeypatch.setattr(tensors, "clause_tensor", bad)
    assert not _contract_pins_hold()


def test_negation_ignored(monkeypatch):
    orig = tensors.clause_tensor
    monkeypatch.setattr(tensors, "clause_tensor", lambda kind, negated: orig(kind, [0] * len(negated)))
    assert not _contract_pins_hold()


def test_copy_rank0_wrong(monkeypatch):
    orig = tensors.copy_tensor
    monkeypatch.setattr(tensors, "copy_tensor", lambda d: np.array(1, dtype=object) if d == 0 else orig(d))
    assert not _contract_pins_hold()


def test_contraction_transposed_operand(monkeypatch):
    orig = contract.contract_pair

    def bad(A, B, p=None):
        t, l = orig(A, B, p)
        if t.ndim >= 2:
            t = np.swapaxes(t, 0, 1)  # labels no longer match the axes
        return t, l
    monkeypatch.setattr(contract, "contract_pair", bad)
    assert not _contract_pins_hold()


def test_modular_product_dropped_term(monkeypatch):
    def bad(A, B, axes, p):
        A = A.astype(np.int64)
        B = B.astype(np.int64)
        a0, a1 = A & 0xFFFF, A >> 16
        b0, b1 = B & 0xFFFF, B >> 16
        s00 = np.tensordot(a0, b0, axes=axes) % p
        s01 = np.tensordot(a0, b1, axes=axes) % p
        s10 = np.tensordot(a1, b0, axes=axes) % p
        mid = (s01 + s10) % p
        return ((mid * ((1 << 16) % p)) % p + s00) % p
    monkeypatch.setattr(contract, "_mod_tensordot", bad)
    assert not _rns_pins_hold()


def test_crt_missing_inverse(monkeypatch):
    def bad(residues, primes):
        M = 1
        for p in primes:
            M *= p
        return sum(r * (M // p) for r, p in zip(residues, primes)) % M
    monkeypatch.setattr(rns, "crt", bad)
    assert not _rns_pins_hold()


def test_elimination_sums_one_value(monkeypatch):
    orig = elim._product

    def bad(factors, p):
        t, scope = orig(factors, p)
        t = t.copy()
        # zero the slice where the lowest variable of the scope is 1
        t[(1,) + (slice(None),) * (t.ndim - 1)] = 0
        return t, scope
    monkeypatch.setattr(elim, "_product", bad)
    f = I.vertex_cover_formula(I.prism_graph(5))
    assert elim.count(f) != 81


def test_brute_force_wrong_or_rule(monkeypatch):
    orig = brute.clause_true_count
    monkeypatch.setattr(brute, "clause_true_count", lambda x, lits: orig(x, lits[:-1]) if lits else orig(x, lits))
    assert brute.count_numpy(I.vertex_cover_formula(I.complete_graph(4))) != 5
