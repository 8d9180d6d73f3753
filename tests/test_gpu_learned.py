"""The trained order scorer against the plain method: on held-out 1-in-3
instances (n in [100, 180], alpha = 0.66) where greedy stays within the rank
cap, counts under the learned order equal the oracle's, and contracting with
the learned orders takes less GPU time in total than with greedy's."""
import os
import time

import pytest

import instances as I
from oracle import elim
from paper_1805_00475_amd import tn

pytestmark = pytest.mark.gpu
MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1805_00475_amd", "models",
                     "order_mlp.npy")
HELDOUT = [1, 4, 6, 9, 12, 15, 16, 18, 22, 23]


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _time_contract(net, plan, reps=3):
    import torch
    tn.count_plan(net, plan)  # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        v = tn.count_plan(net, plan)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps, v


def test_learned_counts_and_gain_over_greedy():
    model = tn.Model.load_file(MODEL)
    tot_g = tot_l = 0.0
    for i in HELDOUT:
        f = I.learned_instance(i, "heldout")
        net = tn.Network(f)
        pg = net.order("greedy")
        pl = net.order("learned_raw", model=model)
        _say(f"held-out {i} n={f.n_vars}: greedy rank {pg.stats['max_rank']}, learned rank {pl.stats['max_rank']}")
        tg, cg = _time_contract(net, pg)
        tl, cl = _time_contract(net, pl)
        want = elim.count_rns(f)
        assert cg == want and cl == want
        tot_g += tg
        tot_l += tl
    _say(f"greedy {1000 * tot_g:.2f} ms, learned {1000 * tot_l:.2f} ms")
    assert tot_l < tot_g
