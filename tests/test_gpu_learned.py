"""The trained order scorer against the plain method, on held-out 1-in-3
instances (alpha = 0.66, n in [100, 250]). The instances are chosen by a
stated rule, computed here: indices i < 64 whose greedy plan fits the rank
cap and is predicted to contract in at most 20 ms; the excluded ones are
printed. Counts under every order equal the oracle's, and ordering plus
contracting with the learned order -- alone, and judged against greedy --
takes less wall time in total than with greedy's."""
import os
import sys
import time

import pytest

import instances as I
from oracle import elim
from paper_1805_00475_amd import tn

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "paper_1805_00475_amd", "models", "order_mlp.npy")


def _say(*a):
    print("[gpu case]", *a, file=sys.stderr, flush=True)


def _instances():
    keep, skip = [], []
    for i in range(64):
        net = tn.Network(I.learned_instance(i, "heldout"))
        try:
            p = net.order("greedy")
        except tn.TNError:
            skip.append(i)
            continue
        (keep if 2 ** p.stats["log2_cost"] <= 20000.0 else skip).append(i)
    return keep, skip


def _wall(net, kind, seed, model, reps=3):
    import torch
    plan = net.order(kind, seed=seed, model=model)
    tn.count_plan(net, plan)  # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        p = net.order(kind, seed=seed, model=model)
        v = tn.count_plan(net, p)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps, v, plan


def test_learned_counts_and_gain_over_greedy():
    model = tn.Model.load_file(MODEL)
    keep, skip = _instances()
    _say(f"held-out instances kept {keep}, excluded {skip}")
    assert len(keep) >= 10
    tot = {"greedy": 0.0, "learned_raw": 0.0, "learned": 0.0}
    fallbacks = 0
    for i in keep:
        f = I.learned_instance(i, "heldout")
        net = tn.Network(f)
        want = elim.count_rns(f)
        for kind in tot:
            t, v, plan = _wall(net, kind, i, model if "learned" in kind else None)
            assert v == want, (i, kind)
            tot[kind] += t
            if kind == "learned":
                fallbacks += plan.stats["fallback"]
        _say(f"held-out {i} n={f.n_vars}: " + ", ".join(f"{k} {1000 * v:.1f}" for k, v in tot.items()))
    _say(f"order + contract totals (ms): " + ", ".join(f"{k} {1000 * v:.2f}" for k, v in tot.items()) +
         f"; learned fallback rate {fallbacks / len(keep):.2f}")
    assert tot["learned_raw"] < tot["greedy"]
    assert tot["learned"] < tot["greedy"]
    assert fallbacks < len(keep)
