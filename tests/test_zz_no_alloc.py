"""tn_contract_noalloc (the library's own file-scope device array as the
workspace) against tn_contract on the same plans: residues and 64-bit counts
bit-identical, on calls in a row whose inputs shrink, plus the size limit."""
import json
import os
import sys

import pytest

import instances as I
from oracle import brute
from paper_1805_00475_amd import tn

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _gold_cvc(n, seed):
    items = json.load(open(os.path.join(GOLD, "cvc_counts.json")))["items"]
    return int(next(it["count"] for it in items if it["n"] == n and it["seed"] == seed))


def _fits(net, plan, **kw):
    return tn.workspace_bytes(net, plan, **kw) <= tn.noalloc_max_bytes()


def test_noalloc_matches_contract_on_shrinking_inputs():
    assert tn.noalloc_max_bytes() == 64 << 20
    # 1: vertex cover n=120, small moduli (int8 planes)
    f1 = I.cvc(120, 0)
    n1 = tn.Network(f1)
    p1 = n1.order("best", seed=0)
    assert _fits(n1, p1)
    _say(f"[gpu] noalloc cvc n=120 s0 max_rank={p1.stats['max_rank']}")
    want = tn.contract(n1, p1)
    got = tn.contract_noalloc(n1, p1)
    assert got == want
    assert tn.crt_moduli(got, tn.moduli(p1)) == _gold_cvc(120, 0)
    # 2: smaller, 16-bit primes (u32 planes, digit-plane matrix cores)
    f2 = I.cvc(60, 1)
    n2 = tn.Network(f2)
    p2 = n2.order("partition", seed=3)
    _say(f"[gpu] noalloc cvc n=60 s1 wide primes max_rank={p2.stats['max_rank']}")
    want = tn.contract(n2, p2, arith="rns", flags=tn.FLAG_WIDE_RNS)
    got = tn.contract_noalloc(n2, p2, arith="rns", flags=tn.FLAG_WIDE_RNS)
    assert got == want
    mods = tn.moduli(p2, arith="rns", flags=tn.FLAG_WIDE_RNS)
    assert min(mods) > 255 and tn.crt_moduli(got, mods) == _gold_cvc(60, 1)
    # 3: smaller again, 64-bit counts
    f3 = I.small_1in3(7)
    n3 = tn.Network(f3)
    p3 = n3.order("greedy")
    _say("[gpu] noalloc 1-in-3 n=20 u64")
    got = tn.contract_noalloc(n3, p3)
    assert got == tn.contract(n3, p3) == brute.count(f3)
    # 4: the first input again after the array held smaller ones
    _say("[gpu] noalloc cvc n=120 s0 again")
    assert tn.crt_moduli(tn.contract_noalloc(n1, p1), tn.moduli(p1)) == _gold_cvc(120, 0)


def test_noalloc_rejects_plans_beyond_the_array():
    f = I.cvc(200, 0)
    net = tn.Network(f)
    plan = net.order("partition", seed=0)
    assert not _fits(net, plan)
    _say(f"[gpu] noalloc too big: cvc n=200 max_rank={plan.stats['max_rank']}")
    with pytest.raises(tn.TNError) as e:
        tn.contract_noalloc(net, plan)
    assert e.value.status == -4   # TN_ETOOBIG, before any device work
    with pytest.raises(tn.TNError) as e:
        tn.contract_noalloc(net, plan, flags=tn.FLAG_TIMING)
    assert e.value.status == -7
