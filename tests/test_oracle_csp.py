"""Pins of the oracle's other clause types and general constraint networks
(parity clauses, 1-in-k, non-boolean domains, integer weights: the
generalisations of Sec. 4) against results fixed outside the oracle:
chromatic polynomials of cycles, complete graphs and paths, the transfer
matrix of the hard-core model, the GF(2) rank formula for #XORSAT, closed
forms of disjoint 1-in-k clauses; enumeration against contraction on random
instances; planted mistakes that must fail a pin."""
import math

import numpy as np
import pytest

import instances as I
from oracle import brute, contract, csp, elim


from oracle.closed import chromatic_complete, chromatic_cycle, hardcore_cycle, xorsat_count  # noqa: E402


def _pins_hold():
    """CSP oracle against the closed forms (both of its computations)."""
    for n, q in ((5, 3), (6, 4), (4, 5)):
        c = I.coloring_csp(I.cycle_graph(n), n, q)
        if csp.count_brute(c) != chromatic_cycle(n, q) or csp.count_contract(c) != chromatic_cycle(n, q):
            return False
    for n, q in ((4, 4), (4, 5), (3, 6)):
        c = I.coloring_csp(I.complete_graph(n), n, q)
        if csp.count_contract(c) != chromatic_complete(n, q) or csp.count_brute(c) != chromatic_complete(n, q):
            return False
    path = [(i, i + 1) for i in range(6)]
    if csp.count_contract(I.coloring_csp(path, 7, 3)) != 3 * 2 ** 6:
        return False
    for n, lam in ((5, 1), (7, 3), (6, 10)):
        c = I.hardcore_csp(I.cycle_graph(n), n, lam)
        if csp.count_brute(c) != hardcore_cycle(n, lam) or csp.count_contract(c) != hardcore_cycle(n, lam):
            return False
    # an asymmetric table, by hand: w1[a][b] = 3a + b over domains 2 x 3, w2 = [1, 10]
    # Z = (0 + 1 + 2) * 1 + (3 + 4 + 5) * 10 = 123
    c = I.CSP(2, [2, 3], [((1, 2), [0, 1, 2, 3, 4, 5]), ((1,), [1, 10])])
    if csp.count_brute(c) != 123 or csp.count_contract(c) != 123:
        return False
    # a proper 3-colouring of one edge (6), an unused variable of domain 4
    # (x4) and a one-value variable with a unary weight 5 (x5): 120
    c = I.CSP(4, [3, 3, 4, 1], [((1, 2), [1 if a != b else 0 for a in range(3) for b in range(3)]),
                               ((4,), [5])])
    if csp.count_contract(c) != 120 or csp.count_brute(c) != 120:
        return False
    return True


def test_closed_forms():
    assert _pins_hold()


def test_large_closed_forms_by_contraction():
    # RNS path of the contractor: counts above 2^62 with weights up to 1000
    assert csp.count_rns(I.coloring_csp(I.cycle_graph(60), 60, 3)) == chromatic_cycle(60, 3)
    assert csp.count_rns(I.coloring_csp(I.cycle_graph(40), 40, 7)) == chromatic_cycle(40, 7)
    assert csp.count_rns(I.hardcore_csp(I.cycle_graph(30), 30, 1000)) == hardcore_cycle(30, 1000)


def test_brute_and_contraction_agree_on_random_csps():
    rng = I.Rng(2024)
    for _ in range(30):
        c = I.random_csp(6, 7, rng, max_domain=4, max_arity=3, max_weight=4)
        want = csp.count_brute(c)
        assert csp.count_contract(c) == want
        assert csp.count_contract(c, p=2147483647) == want % 2147483647


def test_table_csp_of_formula_matches_brute_force():
    rng = I.Rng(77)
    for _ in range(12):
        f = I.random_mixed_formula(8, 7, rng)
        f.clauses = [(k if r < 2 else I.XOR, cl) for (k, cl), r in zip(f.clauses, [rng.below(3) for _ in f.clauses])]
        assert csp.count_brute(I.table_csp(f)) == brute.count_numpy(f)


def test_xorsat_rank_formula():
    rng = I.Rng(5)
    seen_zero = seen_pos = False
    for _ in range(20):
        f = I.xor_k(14, rng.below(16), 3, rng)
        want = xorsat_count(f)
        assert brute.count_numpy(f) == want
        assert brute.count_c(f) == want
        assert elim.count(f) == want
        assert contract.count_exact(f) == want
        seen_zero |= want == 0
        seen_pos |= want > 0
    assert seen_zero and seen_pos


def test_xor_with_repeated_literals_counts_occurrences():
    # x1 XOR x1 is always even: unsatisfiable; x1 XOR -x1 is always odd
    assert brute.count_numpy(I.Formula(2, [(I.XOR, [1, 1])])) == 0
    assert brute.count_c(I.Formula(2, [(I.XOR, [1, -1])])) == 4
    assert contract.count_exact(I.Formula(2, [(I.XOR, [1, -1])])) == 4
    assert brute.count_numpy(I.Formula(3, [(I.XOR, [])])) == 0


def test_disjoint_one_in_k():
    for k in (4, 5, 7):
        n = 3 * k + 2
        f = I.Formula(n, [(I.EXACTLY_ONE, list(range(1 + j * k, 1 + (j + 1) * k))) for j in range(3)])
        assert brute.count_numpy(f) == k ** 3 * 4
        assert contract.count_exact(f) == k ** 3 * 4
    rng = I.Rng(9)
    f = I.exactly_one_k(16, 6, 5, rng)
    assert all(len(set(c)) == 5 for _, c in f.clauses)
    assert brute.count_c(f) == elim.count(f) == contract.count_exact(f)


# ------------------------------------------------------------ planted mistakes
def test_copy_not_diagonal_caught(monkeypatch):
    orig = csp.network

    def bad(c, p=None):
        out = []
        for t, ls in orig(c, p):
            if len(ls) >= 2 and t.ndim == len(ls) and t.ndim >= 2 and t.sum() == t.shape[0] and \
                    all(t[(x,) * t.ndim] == 1 for x in range(t.shape[0])):
                t = t.copy()
                t[(0,) * (t.ndim - 1) + (1,)] = 1   # one off-diagonal entry
            out.append((t, ls))
        return out
    monkeypatch.setattr(csp, "network", bad)
    assert not _pins_hold()


def test_table_read_column_major_caught(monkeypatch):
    orig = csp._table

    def bad(c, scope, table, dtype=object):
        shape = tuple(c.domain[v - 1] for v in scope)
        t = np.array([int(x) for x in table], dtype=dtype)
        return t.reshape(shape, order="F") if shape else t.reshape(())
    monkeypatch.setattr(csp, "_table", bad)
    assert not _pins_hold()


def test_unused_variable_weight_caught(monkeypatch):
    orig = csp.network

    def bad(c, p=None):
        return [(np.array(1, dtype=t.dtype) if (t.ndim == 0 and not ls) else t, ls) for t, ls in orig(c, p)]
    monkeypatch.setattr(csp, "network", bad)
    assert not _pins_hold()


def test_parity_rule_off_by_one_caught(monkeypatch):
    from oracle import tensors
    orig = tensors.clause_tensor

    def bad(kind, negated):
        t = orig(kind, negated)
        if kind == tensors.XOR:
            t = 1 - t                          # even instead of odd
        return t
    monkeypatch.setattr(tensors, "clause_tensor", bad)
    # x1+x2 = x2+x3 = x1+x3 = 1 over GF(2) is inconsistent (the three sum to
    # 0 = 1); with even parity it has 2 solutions
    f = I.Formula(3, [(I.XOR, [1, 2]), (I.XOR, [2, 3]), (I.XOR, [1, 3])])
    assert xorsat_count(f) == 0
    assert contract.count_exact(f) != xorsat_count(f)
