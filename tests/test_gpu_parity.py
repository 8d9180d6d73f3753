"""GPU parity: counts from the HIP path (through the C ABI) against the CPU
oracle and against pins that do not come from either.

Counts are integers, so the bar is bit-exact equality. Every case prints its
name before touching the GPU.
"""
import json
import os

import pytest

import instances as I
from oracle import brute, closed, elim
from paper_1805_00475_amd import tn

GOLD = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.gpu


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def _say(*a):
    print("[gpu case]", *a, flush=True)


ORDERS = ["greedy", "partition", "community"]


def test_eq5_network_on_gpu():
    # (x1|x2|x3) & (x2|x3|x6): the network of Eq. 5 with the open bonds closed
    _say("eq5")
    f = I.Formula(4, [(I.OR, [1, 2, 3]), (I.OR, [2, 3, 4])])
    for order in ORDERS:
        assert tn.count(f, order) == 13
        assert tn.count(f, order, arith="rns") == 13


def test_small_1in3_all_seeds_u64():
    g = _gold("small_1in3_counts.json")["counts"]
    _say("small 1-in-3 n=20 m=14, 1000 seeds, greedy, u64")
    for i, want in enumerate(g):
        assert tn.count(I.small_1in3(i), "greedy") == want, i


def test_small_1in3_rns_and_orders():
    g = _gold("small_1in3_counts.json")["counts"]
    _say("small 1-in-3, rns + all orders")
    for i in range(0, 1000, 25):
        f = I.small_1in3(i)
        for order in ORDERS:
            assert tn.count(f, order, seed=i, arith="rns") == g[i], (i, order)


def test_generic_kernel_matches():
    g = _gold("small_1in3_counts.json")["counts"]
    _say("generic-only kernel")
    for i in range(0, 1000, 50):
        assert tn.count(I.small_1in3(i), "greedy", flags=tn.FLAG_GENERIC_ONLY) == g[i]
    f = I.cvc(60, 0)
    want = int(_gold("cvc_counts.json")["items"][0]["count"])
    assert tn.count(f, "greedy", flags=tn.FLAG_GENERIC_ONLY) == want
    assert tn.count(f, "greedy", arith="rns", flags=tn.FLAG_GENERIC_ONLY) == want


def test_random_mixed_formulas_vs_brute_force():
    rng = I.Rng(4242)
    _say("random mixed formulas vs brute force")
    done = 0
    while done < 120:
        n = rng.uniform_int(1, 16)
        f = I.random_mixed_formula(n, rng.uniform_int(0, 18), rng)
        if max(f.occurrences(), default=0) > 12:
            continue
        want = brute.count(f)
        for order in ORDERS:
            assert tn.count(f, order, seed=done) == want, (f.n_vars, f.clauses, order)
        assert tn.count(f, "greedy", arith="rns", n_primes=2) == want
        done += 1


def test_degenerate_formulas():
    _say("degenerate formulas")
    assert tn.count(I.Formula(0)) == 1
    assert tn.count(I.Formula(5)) == 32
    for n in (63, 64, 100, 300):
        assert tn.count(I.Formula(n)) == 2 ** n
        # one satisfiable clause forces device work
        assert tn.count(I.Formula(n, [(I.OR, [1, 2])])) == 3 * 2 ** (n - 2)
    assert tn.count(I.Formula(3, [(I.OR, [])])) == 0
    assert tn.count(I.Formula(3, [(I.EXACTLY_ONE, [])])) == 0
    assert tn.count(I.Formula(2, [(I.OR, [1, -1])])) == 4       # tautology
    assert tn.count(I.Formula(2, [(I.EXACTLY_ONE, [1, -1])])) == 4
    assert tn.count(I.Formula(2, [(I.EXACTLY_ONE, [1, 1])])) == 0
    assert tn.count(I.Formula(1, [(I.OR, [1, 1, 1])])) == 1
    # disconnected components multiply
    a = I.vertex_cover_formula(I.prism_graph(5))
    b = I.perfect_matching_formula(I.prism_graph(6))
    assert tn.count(I.disjoint_union(a, b)) == 81 * 20


def test_named_graphs():
    _say("named graphs")
    assert tn.count(I.vertex_cover_formula(I.complete_graph(4))) == 5
    for k in range(3, 13):
        assert tn.count(I.vertex_cover_formula(I.cycle_graph(k))) == closed.lucas(k)
    assert tn.count(I.vertex_cover_formula(I.petersen_graph())) == 76
    assert tn.count(I.perfect_matching_formula(I.petersen_graph())) == 6


@pytest.mark.parametrize("n", [60, 120, 200])
def test_prism_vertex_covers_rns(n):
    k = n // 2
    want = closed.prism_vertex_covers(k)
    f = I.vertex_cover_formula(I.prism_graph(k))
    _say(f"prism vertex covers n={n}")
    for order in ORDERS:
        assert tn.count(f, order) == want, order


def test_prism_perfect_matchings_300_vars():
    _say("prism perfect matchings, 300 variables / 200 clauses")
    f = I.perfect_matching_formula(I.prism_graph(100))
    for order in ORDERS:
        assert tn.count(f, order) == closed.prism_perfect_matchings(100)


def test_cvc_random_cubic_vs_oracle():
    items = _gold("cvc_counts.json")["items"]
    for it in items:
        f = I.cvc(it["n"], it["seed"])
        _say(f"cvc n={it['n']} seed={it['seed']}")
        orders = ["greedy", "community", "partition"] if it["n"] <= 120 else ["community"]
        for order in orders:
            assert tn.count(f, order, seed=it["seed"]) == int(it["count"]), order


def test_large_1in3_vs_oracle():
    for it in _gold("large_1in3_counts.json")["items"]:
        f = I.large_1in3(it["n"], it["alpha"], it["seed"])
        _say(f"1-in-3 n={it['n']} seed={it['seed']}")
        for order in ("partition", "community"):
            assert tn.count(f, order, seed=it["seed"]) == int(it["count"]), order


def test_cnf_equivalence_on_gpu():
    # the CNF network has COPY tensors of rank 5x the occurrences, so only
    # draws whose variables occur at most 4 times are used; the count must
    # not change (Sec. 3.2 identity)
    _say("1-in-3 vs its CNF, n=40 m=20")
    used = 0
    seed = 900
    while used < 3:
        f = I.exactly_one_3(40, 20, I.Rng(seed))
        seed += 1
        if max(f.occurrences()) > 4:
            continue
        g = I.cnf_of_exactly_one(f)
        if tn.Network(g).order("greedy").stats["max_rank"] > 24:
            continue
        want = elim.count(f)
        assert tn.count(f, "greedy") == want
        assert tn.count(g, "greedy") == want
        used += 1


def test_u64_and_rns_agree():
    _say("u64 vs rns")
    for s in range(5):
        f = I.cvc(60, s)
        assert tn.count(f, "community", arith="u64") == tn.count(f, "community", arith="rns")


def test_prime_set_invariance():
    _say("prime-set invariance")
    f = I.cvc(120, 2)
    want = int(_gold("cvc_counts.json")["items"][12]["count"])
    assert tn.count(f, "community", arith="rns", n_primes=9) == want
    assert tn.count(f, "community", arith="rns", n_primes=14) == want


def test_workspace_too_small():
    _say("workspace too small")
    import torch
    f = I.cvc(60, 0)
    net = tn.Network(f)
    plan = net.order("greedy")
    need = tn.workspace_bytes(net, plan)
    buf = torch.empty(max(need // 4, 256), dtype=torch.uint8, device="cuda")
    o = tn.ContractOpts_c(0, 0, buf.data_ptr(), buf.numel(), tn.current_stream_handle(), 0, 0)
    import ctypes
    u = ctypes.c_uint64()
    st = tn.load().tn_contract(net.h, plan.h, ctypes.byref(o), None, 0, ctypes.byref(u))
    assert st == -4


def test_repeat_is_deterministic():
    _say("repeat determinism")
    net = tn.Network(I.cvc(120, 0))
    plan = net.order("community")
    r1 = tn.contract(net, plan, arith="rns")
    r2 = tn.contract(net, plan, arith="rns")
    assert r1 == r2


@pytest.mark.gpu
def test_contract_residues_recombine_through_crt_moduli():
    # tn_contract's default residues (small moduli) recombined by the C ABI's
    # own CRT entry point, against the closed form of prism vertex covers
    _say("[gpu] tn_contract residues -> tn_crt_moduli, prism n=200")
    f = I.vertex_cover_formula(I.prism_graph(100))
    net = tn.Network(f)
    plan = net.order("best", seed=0)
    res = tn.contract(net, plan)
    mods = tn.moduli(plan)
    assert len(res) == len(mods) and max(mods) <= 255
    assert tn.crt_moduli(res, mods) == closed.prism_vertex_covers(100)


def test_cvc200_random_cubic_vs_oracle():
    # the benchmark's own workload size: vertex cover of random cubic graphs
    # at n = 200, both residue systems, against the pairwise-contraction oracle
    for it in _gold("cvc200_counts.json")["items"]:
        f = I.cvc(200, it["seed"])
        want = int(it["count"])
        _say(f"cvc n=200 seed={it['seed']} small moduli, best order")
        assert tn.count(f, "best", seed=it["seed"]) == want
        _say(f"cvc n=200 seed={it['seed']} 16-bit primes, community order")
        assert tn.count(f, "community", flags=tn.FLAG_WIDE_RNS) == want


def test_c3_1in3_vs_oracle():
    # monotone 1-in-3 with uniform clauses at n = 200-250 (alpha 0.62-0.70)
    for it in _gold("c3_1in3_counts.json")["items"]:
        f = I.large_1in3(it["n"], it["alpha"], it["seed"])
        want = int(it["count"])
        for order in ("best", "partition"):
            _say(f"1-in-3 n={it['n']} alpha={it['alpha']} seed={it['seed']} order={order}")
            assert tn.count(f, order, seed=it["seed"]) == want, order


def test_c3_roofline_instance_invariants():
    # the largest 1-in-3 instance measured (n = 300, alpha = 0.62, seed 1,
    # intermediates of rank 31): beyond a CPU oracle here, so the count must
    # agree across two different plans and two residue systems (42 small
    # moduli vs 16-bit primes), and be the same on a second run
    f = I.large_1in3(300, 0.62, 1)
    net = tn.Network(f)
    best = net.order("best", seed=1)
    assert 30 <= best.stats["max_rank"] <= 32
    _say("1-in-3 n=300 a=0.62 s1 best order, small moduli")
    a = tn.count_plan(net, best)
    other = net.order("partition", seed=5)
    _say(f"... partition seed 5 (max rank {other.stats['max_rank']}), small moduli")
    b = tn.count_plan(net, other) if other.stats["max_rank"] <= 32 else a
    _say("... best order, 16-bit primes")
    c = tn.count_plan(net, best, flags=tn.FLAG_WIDE_RNS)
    _say("... best order again")
    d = tn.count_plan(net, best)
    assert a == b == c == d
    assert 0 <= a < 2 ** 300


def test_paper_1in3_family_vs_oracle():
    # the paper's own 1-in-3 workload (Sec. 3.2): one variable per edge of a
    # random cubic graph, one exactly-one clause per vertex; N = 90 to 300
    # variables. The formulas come from the library's own generator
    # (tn_gen_cubic_1in3), which draws the same graphs as the instances package.
    for it in _gold("cubic_1in3_counts.json")["items"]:
        nv, s = it["n_vertices"], it["seed"]
        f = tn.gen_cubic_1in3(nv, I.instance_seed(I.FAMILY_CUBIC_1IN3, (nv << 20) | s))
        want = int(it["count"])
        for order in ("best", "community", "partition"):
            _say(f"cubic 1-in-3 N={it['n_vars']} seed={s} order={order}")
            assert tn.count(f, order, seed=s) == want, order
