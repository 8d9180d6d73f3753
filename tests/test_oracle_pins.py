"""Pins of the CPU oracle against values that do not come from the oracle.

* the worked example of Eq. 5 (Sec. 2.1), stored in tests/golden;
* counts with a plain combinatorial meaning (vertex covers, perfect
  matchings) recomputed by brute force, and closed forms checked by brute
  force on small sizes;
* invariants: empty formula 2^n, disjoint unions multiply, a variable in no
  clause doubles the count, the 1-in-3 <-> 5-clause CNF identity of Sec. 3.2,
  order invariance and prime-set invariance (Sec. 2.1, CRT uniqueness);
* agreement of three independent algorithms (brute force, pairwise
  contraction, bucket elimination) on random mixed formulas.
"""
import itertools
import json
import os
import random

import numpy as np
import pytest

import instances as I
from oracle import brute, closed, contract, cost, elim, rns, tensors

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


# ---------------------------------------------------------------- Eq. 5
def test_eq5_worked_example():
    g = _gold("eq5_worked_example.json")
    net = []
    for t in g["tensors"]:
        d = len(t["labels"])
        arr = tensors.copy_tensor(d) if t["kind"] == "COPY" else tensors.clause_tensor(0, [0] * d)
        net.append((arr, tuple(t["labels"])))
    out = contract.contract_network(net)
    assert len(out) == 1
    arr, labels = out[0]
    assert tuple(sorted(labels)) == tuple(g["open_labels"])
    if labels != tuple(g["open_labels"]):
        arr = arr.T
    assert arr.tolist() == g["result"]
    # every other order of the same four tensors gives the same open tensor
    for order in ([(0, 1), (2, 3), (4, 5)], [(1, 3), (0, 2), (4, 5)], [(2, 3), (1, 4), (0, 5)]):
        (arr2, l2), = contract.contract_network(net, order)
        if l2 != tuple(g["open_labels"]):
            arr2 = arr2.T
        assert arr2.tolist() == g["result"]


def test_eq5_closed_sum():
    # closing the two open bonds sums the four entries: 3+3+3+4 = 13, which
    # brute force over the two-clause formula (x1|x2|x3)&(x2|x3|x6) confirms
    f = I.Formula(4, [(I.OR, [1, 2, 3]), (I.OR, [2, 3, 4])])
    assert brute.count(f) == 13


# --------------------------------------------------------- tensor entries
def test_tensor_entries_against_brute_force_on_single_clauses():
    # a single clause over distinct variables: the clause tensor's entry sum
    # equals the brute-force count of the one-clause formula
    for kind in (I.OR, I.EXACTLY_ONE):
        for d in range(0, 5):
            for neg in itertools.product((0, 1), repeat=d):
                lits = [(-(k + 1) if neg[k] else (k + 1)) for k in range(d)]
                f = I.Formula(d, [(kind, lits)])
                t = tensors.clause_tensor(kind, list(neg))
                assert int(np.sum(t)) == brute.count(f)


def test_copy_tensor_counts_one_variable():
    # a variable alone contributes 2 assignments, whatever its occurrence count
    for d in range(0, 6):
        assert int(np.sum(tensors.copy_tensor(d))) == 2


# ----------------------------------------------------------- brute force
def test_empty_formula_is_two_to_the_n():
    for n in range(0, 21):
        assert brute.count_numpy(I.Formula(n)) == 2 ** n
    assert brute.count_c(I.Formula(26)) == 2 ** 26


def test_empty_clause_gives_zero():
    for kind in (I.OR, I.EXACTLY_ONE):
        f = I.Formula(3, [(I.OR, [1, 2]), (kind, [])])
        assert brute.count(f) == 0
        assert contract.count_exact(f) == 0
        assert elim.count(f) == 0


def test_named_graph_counts():
    g = _gold("closed_form_pins.json")
    assert brute.count(I.vertex_cover_formula(I.complete_graph(4))) == g["k4_vertex_covers"]["value"]
    assert brute.count(I.vertex_cover_formula(I.complete_bipartite_graph(3, 3))) == g["k33_vertex_covers"]["value"]
    assert brute.count(I.vertex_cover_formula(I.petersen_graph())) == g["petersen_vertex_covers"]["value"]
    assert brute.count(I.vertex_cover_formula(I.cube_graph())) == g["q3_vertex_covers"]["value"]
    assert brute.count(I.perfect_matching_formula(I.complete_graph(4))) == g["k4_perfect_matchings"]["value"]
    assert brute.count(I.perfect_matching_formula(I.complete_bipartite_graph(3, 3))) == g["k33_perfect_matchings"]["value"]
    assert brute.count(I.perfect_matching_formula(I.petersen_graph())) == g["petersen_perfect_matchings"]["value"]
    assert brute.count(I.perfect_matching_formula(I.cube_graph())) == g["q3_perfect_matchings"]["value"]


def test_cycles_are_lucas_numbers():
    g = _gold("closed_form_pins.json")["cycle_vertex_covers"]
    for k, v in zip(g["k"], g["value"]):
        assert brute.count(I.vertex_cover_formula(I.cycle_graph(k))) == v
        assert closed.cycle_vertex_covers(k) == v


def test_complete_bipartite_closed_form():
    for a in range(1, 6):
        for b in range(1, 6):
            f = I.vertex_cover_formula(I.complete_bipartite_graph(a, b))
            assert brute.count(f) == closed.complete_bipartite_vertex_covers(a, b)


def test_prism_closed_forms_against_brute_force():
    g = _gold("closed_form_pins.json")
    for k, v in zip(g["prism_vertex_covers"]["k"], g["prism_vertex_covers"]["value"]):
        assert closed.prism_vertex_covers(k) == v
        if 2 * k <= 20:
            assert brute.count(I.vertex_cover_formula(I.prism_graph(k))) == v
    for k, v in zip(g["prism_perfect_matchings"]["k"], g["prism_perfect_matchings"]["value"]):
        assert closed.prism_perfect_matchings(k) == v
        if 3 * k <= 24:
            assert brute.count(I.perfect_matching_formula(I.prism_graph(k))) == v


def test_disjoint_1in3_closed_form():
    for m in range(0, 5):
        for extra in range(0, 4):
            n = 3 * m + extra
            f = I.Formula(n, [(I.EXACTLY_ONE, [3 * i + 1, 3 * i + 2, 3 * i + 3]) for i in range(m)])
            assert brute.count(f) == closed.disjoint_1in3(n, m)


def test_numpy_and_c_brute_force_agree():
    rng = I.Rng(12345)
    for _ in range(40):
        n = rng.uniform_int(1, 14)
        f = I.random_mixed_formula(n, rng.uniform_int(0, 12), rng)
        assert brute.count_numpy(f) == brute.count_c(f)


# ----------------------------------------------------------- invariants
def test_cnf_equivalence_of_1in3():
    # Sec. 3.2: a monotone 1-in-3 clause equals five OR clauses with negations
    for i in range(30):
        f = I.small_1in3(i)
        g = I.cnf_of_exactly_one(f)
        assert brute.count(f) == brute.count(g)
        assert elim.count(f) == elim.count(g)
    rng = I.Rng(31)
    for _ in range(10):
        f = I.exactly_one_3(9, 4, rng)
        g = I.cnf_of_exactly_one(f)
        assert contract.count_exact(f) == contract.count_exact(g) == brute.count(f)


def test_disjoint_union_multiplies():
    rng = I.Rng(7)
    for _ in range(10):
        a = I.random_mixed_formula(6, 5, rng)
        b = I.random_mixed_formula(7, 6, rng)
        u = I.disjoint_union(a, b)
        assert contract.count_exact(u) == contract.count_exact(a) * contract.count_exact(b)
        assert brute.count(u) == brute.count(a) * brute.count(b)


def test_unused_variable_doubles():
    f = I.small_1in3(3)
    g = I.Formula(f.n_vars + 2, list(f.clauses))
    assert contract.count_exact(g) == 4 * contract.count_exact(f)
    assert elim.count(g) == 4 * elim.count(f)


# ------------------------------------------- three algorithms must agree
def _random_formulas(seed, count, nmax=12, max_occ=7):
    """Random mixed formulas; draws in which a variable occurs more than
    ``max_occ`` times are redrawn so the COPY tensors stay small."""
    rng = I.Rng(seed)
    made = 0
    while made < count:
        n = rng.uniform_int(0, nmax)
        m = rng.uniform_int(0, 14)
        if n == 0:
            f = I.Formula(0, [(rng.below(2), []) for _ in range(rng.below(2))])
        else:
            f = I.random_mixed_formula(n, m, rng)
        if max(f.occurrences(), default=0) > max_occ:
            continue
        made += 1
        yield f


def test_contractor_and_elimination_match_brute_force():
    for f in _random_formulas(2024, 150):
        want = brute.count(f)
        assert contract.count_exact(f) == want, f.clauses
        assert elim.count(f) == want, f.clauses
        assert contract.count_rns(f) == want
        assert elim.count_rns(f) == want


def test_config1_all_three_agree():
    for i in range(0, 1000, 37):
        f = I.small_1in3(i)
        want = brute.count_c(f)
        assert contract.count_exact(f) == want
        assert elim.count(f) == want


def test_order_invariance():
    # any valid pairwise order gives the same count (Sec. 2.1)
    rnd = random.Random(5)
    for f in _random_formulas(99, 25, nmax=10):
        nets, _ = tensors.network_of_formula(f)
        labels = [set(ls) for _, ls in nets]
        want = contract.count_exact(f)
        for _ in range(3):
            live = dict(enumerate(labels))
            nid = len(labels)
            order = []
            while len(live) > 1:
                i, j = sorted(rnd.sample(sorted(live), 2))
                live[nid] = live.pop(i) ^ live.pop(j)
                order.append((i, j))
                nid += 1
            assert contract.count_exact(f, order) == want


def test_prime_set_invariance():
    f = I.cvc(24, 3)
    want = brute.count(f)
    p1 = rns.largest_primes_below(1 << 31, 3)
    p2 = rns.largest_primes_below(1 << 31, 7)[4:]
    assert contract.count_rns(f, p1) == want
    assert contract.count_rns(f, p2) == want
    assert elim.count_rns(f, p2) == want


# -------------------------------------------------------------- residues
def _miller_rabin(q):
    if q < 2:
        return False
    d, r = q - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in (2, 3, 5, 7, 11, 13, 17):
        if a % q == 0:
            continue
        x = pow(a, d, q)
        if x in (1, q - 1):
            continue
        for _ in range(r - 1):
            x = x * x % q
            if x == q - 1:
                break
        else:
            return False
    return True


def test_prime_table_is_prime_and_descending():
    ps = rns.largest_primes_below(1 << 31, 16)
    assert all(_miller_rabin(p) for p in ps)
    assert ps == sorted(ps, reverse=True)
    # no prime is skipped between consecutive entries
    for a, b in zip(ps, ps[1:]):
        assert not any(_miller_rabin(q) for q in range(b + 1, a))
    assert ps[0] == 2 ** 31 - 1


def test_prime_count_bound():
    table = rns.largest_primes_below(1 << 31, rns.n_primes_for(1000))
    for n in range(0, 1000, 7):
        k = rns.n_primes_for(n)
        prod = 1
        for p in table[:k]:
            prod *= p
        assert prod > 2 ** n


def test_crt_roundtrip():
    r = random.Random(1)
    ps = rns.largest_primes_below(1 << 31, 11)
    M = 1
    for p in ps:
        M *= p
    for _ in range(200):
        x = r.randrange(M)
        assert rns.crt([x % p for p in ps], ps) == x


# ------------------------------------------------------------ cost replay
def test_cost_replay_on_eq5_network():
    labels = [(1, 2, 3), (2, 4), (3, 5), (4, 5, 6)]
    rep = cost.replay(labels, [(0, 1), (2, 4), (3, 5)])
    # OR(1,2,3)*COPY(2,4) -> {1,3,4}; COPY(3,5)*{1,3,4} -> {1,4,5}; *OR(4,5,6) -> {1,6}
    assert [(s["rA"], s["rB"], s["s"], s["rC"]) for s in rep["steps"]] == [(3, 2, 1, 3), (2, 3, 1, 3), (3, 3, 2, 2)]
    assert rep["max_rank"] == 3
    assert rep["macs"] == 2 ** 4 + 2 ** 4 + 2 ** 4
    assert rep["remaining"] == [[1, 6]]


# ---------------------------------------------------------- generators
def test_generators_are_deterministic_and_well_formed():
    assert I.small_1in3(5).clauses == I.small_1in3(5).clauses
    f = I.small_1in3(11)
    assert f.n_vars == 20 and f.n_clauses == 14
    for kind, cl in f.clauses:
        assert kind == I.EXACTLY_ONE and len(set(cl)) == 3 and all(1 <= v <= 20 for v in cl)
    for n in (60, 120, 200):
        g = I.cvc(n, 0)
        assert g.n_vars == n and g.n_clauses == 3 * n // 2
        assert g.occurrences() == [3] * n
        edges = {tuple(sorted(c)) for _, c in g.clauses}
        assert len(edges) == g.n_clauses
    b = [I.batch_instance(i) for i in range(8)]
    for i, f in enumerate(b):
        assert 30 <= f.n_vars <= 120
        if i % 2:
            assert f.n_vars % 2 == 0 and f.occurrences() == [3] * f.n_vars


def test_rng_bounded_draws_are_uniform_enough():
    rng = I.Rng(42)
    counts = [0] * 6
    for _ in range(60000):
        counts[rng.below(6)] += 1
    assert max(counts) - min(counts) < 600


def test_step_definition_matches_pairwise_contraction():
    # the entry-by-entry step definition agrees with labelled tensordot
    rng = np.random.default_rng(1)
    p = 2147483647
    for rA, rB, s, maskA in ((5, 4, 2, 0b10110), (6, 6, 3, 0b100101), (4, 2, 0, 0b011110), (3, 3, 3, 0)):
        rC = rA + rB - 2 * s
        A = rng.integers(0, p, 1 << rA)
        B = rng.integers(0, p, 1 << rB)
        la = tuple(("z", k) if k < s else ("a", k - s) for k in reversed(range(rA)))
        lb = tuple(("z", k) if k < s else ("b", k - s) for k in reversed(range(rB)))
        Ct, lc = contract.contract_pair((A.reshape((2,) * rA).astype(np.int64), la),
                                        (B.reshape((2,) * rB).astype(np.int64), lb), p)
        ka = kb = 0
        cl = []
        for j in range(rC):
            if (maskA >> j) & 1:
                cl.append(("a", ka))
                ka += 1
            else:
                cl.append(("b", kb))
                kb += 1
        Cf = np.transpose(Ct, [lc.index(l) for l in reversed(cl)]).reshape(-1) if rC else Ct.reshape(-1)
        want = contract.step_entries(A, B, s, maskA, rC, range(1 << rC), p)
        assert [int(x) for x in Cf] == want


def test_mod_tensordot_chunked_shared_dimension_exact():
    # a shared dimension of 2^22 (two float64 chunks of 2^21) against exact
    # Python integers, entries uniform below the largest 31-bit prime
    import numpy as np
    from oracle import contract as C
    r = np.random.default_rng(1)
    p = 2147483647
    A = r.integers(0, p, size=(2,) * 23, dtype=np.int64)
    B = r.integers(0, p, size=(2,) * 23, dtype=np.int64)
    got = C._mod_tensordot(A, B, (list(range(1, 23)), list(range(1, 23))), p)
    a, b = A.reshape(2, -1).tolist(), B.reshape(2, -1).tolist()
    want = [[sum(x * y for x, y in zip(a[i], b[j])) % p for j in range(2)] for i in range(2)]
    assert got.tolist() == want


def test_oracle_orders_valid_and_count_exact():
    # the oracle's own bisection and Girvan-Newman orders merge every tensor
    # exactly once, and O-B along them gives the brute-force count
    from oracle import contract as C, order as O, tensors as T, brute as Bf, cost
    rng = I.Rng(4242)
    forms = [I.random_mixed_formula(9, 8, rng) for _ in range(6)] + \
        [I.vertex_cover_formula(I.petersen_graph()), I.perfect_matching_formula(I.prism_graph(5)),
         I.small_1in3(3), I.Formula(3)]
    for f in forms:
        nets, _ = T.network_of_formula(f)
        labels = [ls for _, ls in nets]
        for merges in (O.partition_order(labels, 1, tries=3), O.community_order(labels),
                       O.cheapest_order(labels, tries=2)[0]):
            used = set()
            for k, (a, b) in enumerate(merges):
                assert a != b and a not in used and b not in used and max(a, b) < len(labels) + k
                used.update((a, b))
            if labels:
                assert len(merges) == len(labels) - 1
                assert cost.replay(labels, merges)["remaining"] == [[]]
            assert C.count_exact(f, merges) == Bf.count(f)
