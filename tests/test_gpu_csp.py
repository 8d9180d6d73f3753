"""GPU parity of the generalisations of Sec. 4 against the oracle: parity
(#XORSAT) and 1-in-k clauses, degree reduction (COPY rings, split clauses),
and weighted constraint networks over any domains -- counts through the C ABI
against brute force, the oracle's native-dimension contraction and closed
forms (chromatic polynomials, the hard-core transfer matrix, the GF(2) rank
formula)."""
import sys

import pytest

import instances as I
from oracle import brute, closed, csp, elim
from paper_1805_00475_amd import tn

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, file=sys.stderr, flush=True)


def test_xorsat_small_vs_brute_force():
    rng = I.Rng(31)
    for _ in range(10):
        f = I.xor_k(22, rng.below(26), 3, rng)
        _say(f"k-XOR n=22 m={f.n_clauses}")
        want = brute.count_c(f)
        assert want == closed.xorsat_count(f)
        for order in ("greedy", "partition"):
            assert tn.count(f, order) == want


@pytest.mark.parametrize("n,k,ms", [(80, 3, (40, 64)), (150, 3, (90, 120)), (120, 5, (30, 40))])
def test_xorsat_rank_formula_rns(n, k, ms):
    # densities up to 0.8 clauses per variable: largest ranks 8 to 28
    rng = I.Rng(n + k)
    for m in ms:
        f = I.xor_k(n, m, k, rng)
        _say(f"k-XOR n={n} k={k} m={m}")
        want = closed.xorsat_count(f)
        assert tn.count(f, "best") == want
        assert tn.count(f, "best", build_flags=tn.BUILD_SPLIT_CLAUSES) == want


@pytest.mark.parametrize("k", [4, 5, 6, 8])
def test_one_in_k(k):
    rng = I.Rng(100 + k)
    for _ in range(4):
        f = I.exactly_one_k(24, 5, k, rng)
        _say(f"1-in-{k} n=24")
        want = brute.count_c(f)
        assert tn.count(f, "greedy") == want
        assert tn.count(f, "greedy", build_flags=tn.BUILD_SPLIT_CLAUSES) == want
    # elimination widths 6, 9, 12 and 20 for k = 4, 5, 6, 8: the oracle stays quick
    f = I.exactly_one_k(80, 16, k, I.Rng(1000 + k))
    _say(f"1-in-{k} n=80 m=16")
    want = elim.count_rns(f)
    assert tn.count(f, "best") == want


def test_degree_reduction_rings_and_chains():
    # variables of high occurrence (COPY rings) and long mixed clauses (chains)
    rng = I.Rng(8)
    for _ in range(6):
        f = I.random_mixed_formula(16, 14, rng, max_len=7)
        f.clauses = [(k if rng.below(3) else I.XOR, c) for k, c in f.clauses]
        want = brute.count_numpy(f)
        net = tn.Network(f, tn.BUILD_RING_COPY | tn.BUILD_SPLIT_CLAUSES)
        assert net.ranks()[0] <= 3
        _say(f"degree-reduced mixed formula n=16, {net.info()[0]} tensors")
        assert tn.count(f, "greedy", build_flags=tn.BUILD_RING_COPY | tn.BUILD_SPLIT_CLAUSES) == want
        assert tn.count(f, "community", build_flags=tn.BUILD_RING_COPY) == want
    # 1-in-3 with many occurrences per variable (COPY tensors of rank up to ~12)
    f = I.exactly_one_3(24, 40, I.Rng(3))
    want = brute.count_c(f)
    assert tn.count(f, "greedy", build_flags=tn.BUILD_RING_COPY) == want
    # cubic vertex cover n=120: every COPY has rank 3, nothing changes
    g = I.cvc(120, 1)
    assert tn.Network(g, tn.BUILD_RING_COPY).info() == tn.Network(g).info()


def test_random_csps_vs_brute_force():
    rng = I.Rng(2718)
    for _ in range(16):
        c = I.random_csp(7, 8, rng, max_domain=6, max_arity=3, max_weight=9)
        want = csp.count_brute(c)
        _say(f"random CSP domains {c.domain}")
        assert tn.count(c, "greedy") == want
        assert tn.count(c, "partition", seed=1) == want


def test_csp_weights_beyond_a_byte_and_wide_primes():
    # weights up to 2^20: the initial tensors are reduced per residue plane
    rng = I.Rng(99)
    for _ in range(6):
        c = I.random_csp(8, 10, rng, max_domain=5, max_arity=3, max_weight=1 << 20)
        want = csp.count_brute(c)
        _say(f"weighted CSP, count of {want.bit_length()} bits")
        assert tn.count(c, "greedy") == want
        assert tn.count(c, "greedy", arith="rns", flags=tn.FLAG_WIDE_RNS) == want
        assert tn.count(c, "greedy", arith="rns") == want


@pytest.mark.parametrize("n,q", [(100, 3), (64, 5), (40, 7), (30, 16)])
def test_cycle_colourings(n, q):
    c = I.coloring_csp(I.cycle_graph(n), n, q)
    _say(f"{q}-colourings of C_{n}")
    for order in ("greedy", "best"):
        assert tn.count(c, order) == closed.chromatic_cycle(n, q)


def test_complete_and_petersen_colourings():
    assert tn.count(I.coloring_csp(I.complete_graph(6), 6, 7)) == closed.chromatic_complete(6, 7)
    # Petersen graph: the oracle's native contraction
    c = I.coloring_csp(I.petersen_graph(), 10, 3)
    assert tn.count(c, "greedy") == csp.count_contract(c) == 120


@pytest.mark.parametrize("n,lam", [(60, 1000), (100, 3), (40, 1 << 30)])
def test_hardcore_cycles(n, lam):
    c = I.hardcore_csp(I.cycle_graph(n), n, lam)
    _say(f"hard-core C_{n} lambda={lam}")
    assert tn.count(c, "greedy") == closed.hardcore_cycle(n, lam)
    assert tn.count(c, "community", flags=tn.FLAG_WIDE_RNS, arith="rns") == closed.hardcore_cycle(n, lam)


def test_colourings_of_random_cubic_graphs_vs_oracle():
    # 3-colourings of cubic graphs n=40: domain 3 (2 bonds per occurrence,
    # code 3 excluded), the oracle contracting in dimension 3
    for s in range(3):
        edges = I.cubic_graph(40, I.Rng(500 + s))
        c = I.coloring_csp(edges, 40, 3)
        _say(f"3-colourings of a cubic graph n=40 seed {s}")
        assert tn.count(c, "best") == csp.count_rns(c)
