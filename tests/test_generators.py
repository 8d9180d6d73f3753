"""The library's seeded generators (tn_gen_*, tn_instance_seed) against the
Python generators of the ``instances`` package: both implement the same
published definitions (SplitMix64 seeding xoshiro256**, rejection for bounded
draws, the configuration model with rejection), so every formula must be
identical, literal for literal."""
import pytest

import instances as I
from instances import gen as G
from paper_1805_00475_amd import tn


def _same(a, b):
    assert a.n_vars == b.n_vars
    assert [(int(k), [int(x) for x in c]) for k, c in a.clauses] == \
        [(int(k), [int(x) for x in c]) for k, c in b.clauses]


@pytest.mark.parametrize("family,index,master", [(0, 0, 0), (1, 5, 0), (3, 77, 9), (5, (200 << 20) | 3, 0)])
def test_instance_seed(family, index, master):
    assert tn.instance_seed(family, index, master) == I.instance_seed(family, index, master)


@pytest.mark.parametrize("n", [4, 6, 20, 60, 200])
def test_cubic_graph(n):
    for s in range(3):
        seed = I.instance_seed(G.FAMILY_CVC, (n << 20) | s)
        assert tn.gen_cubic_graph(n, seed) == I.cubic_graph(n, I.Rng(seed))


def test_named_workloads():
    for i in range(20):
        seed = I.instance_seed(G.FAMILY_SMALL_1IN3, i)
        _same(tn.gen_exactly_one_3(20, 14, seed), I.small_1in3(i))
    for n in (60, 120, 200):
        for s in range(2):
            _same(tn.gen_cubic_vc(n, I.instance_seed(G.FAMILY_CVC, (n << 20) | s)), I.cvc(n, s))
    for n, a in ((150, 0.66), (200, 0.62), (300, 0.70)):
        seed = I.instance_seed(G.FAMILY_LARGE_1IN3, (n << 24) | (int(round(a * 100)) << 16) | 1)
        _same(tn.gen_exactly_one_3(n, int(round(a * n)), seed), I.large_1in3(n, a, 1))
    for nv in (8, 100, 200):
        _same(tn.gen_cubic_1in3(nv, I.instance_seed(G.FAMILY_CUBIC_1IN3, (nv << 20) | 2)), I.cubic_1in3(nv, 2))


def test_generator_errors():
    with pytest.raises(tn.TNError):
        tn.gen_cubic_graph(5, 1)   # odd
    with pytest.raises(tn.TNError):
        tn.gen_cubic_graph(2, 1)
    with pytest.raises(tn.TNError):
        tn.gen_exactly_one_3(2, 1, 1)


def test_generated_formula_builds():
    f = tn.gen_cubic_1in3(20, 7)
    net = tn.Network(f)
    assert net.info() == (30 + 20, 60)


@pytest.mark.parametrize("n", [4, 6, 20, 100])
def test_planar_cubic_graphs(n):
    for s in range(3):
        e = I.planar_cubic_graph(n, I.Rng(1000 * n + s))
        assert len(e) == 3 * n // 2 and len(set(e)) == len(e) and all(a < b for a, b in e)
        deg = [0] * n
        adj = [[] for _ in range(n)]
        for a, b in e:
            deg[a] += 1
            deg[b] += 1
            adj[a].append(b)
            adj[b].append(a)
        assert deg == [3] * n
        seen, stack = {0}, [0]
        while stack:
            for u in adj[stack.pop()]:
                if u not in seen:
                    seen.add(u)
                    stack.append(u)
        assert len(seen) == n   # the dual of a triangulation is connected
