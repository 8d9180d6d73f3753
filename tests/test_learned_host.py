"""Host-side checks of the learned order: features and labels of the
library's traces against the oracle's recomputation, the host forward pass
against float64, validity of learned orders and the judge's fallback."""
import os

import numpy as np
import pytest

import instances as I
from oracle import cost, mlp, tensors
from paper_1805_00475_amd import tn

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1805_00475_amd", "models",
                     "order_mlp.npy")


def _labels(f):
    nets, _ = tensors.network_of_formula(f)
    return [ls for _, ls in nets]


@pytest.mark.parametrize("make", [lambda: I.small_1in3(4), lambda: I.cvc(24, 1), lambda: I.batch_instance(2)])
def test_trace_matches_oracle(make):
    f = make()
    net = tn.Network(f)
    teacher = net.order("partition", seed=1)
    X, lab, g = tn.trace(net, teacher)
    want = mlp.trace(_labels(f), teacher.steps())
    assert len(g) - 1 == len(want)
    for k, rows in enumerate(want):
        a, b = g[k], g[k + 1]
        got = sorted((tuple(np.round(X[i], 6)), int(lab[i])) for i in range(a, b))
        exp = sorted((tuple(np.round(r[1].astype(np.float32), 6)), r[2]) for r in rows)
        assert got == exp, k
    # every state has at least one positive (the teacher's own merge)
    assert all(lab[g[k]:g[k + 1]].any() for k in range(len(g) - 1))


def test_host_score_matches_float64():
    p = mlp.init_params(11).astype(np.float32)
    m = tn.Model(p)
    assert np.array_equal(m.params(), p)
    x = np.random.default_rng(2).normal(0, 1, (300, 10)).astype(np.float32)
    got = m.score(x)
    want, _, _ = mlp.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.allclose(got, want, rtol=1e-4, atol=1e-4 * np.abs(want).max())


def test_learned_orders_are_valid():
    m = tn.Model(mlp.init_params(3).astype(np.float32))
    for f in [I.small_1in3(1), I.cvc(60, 2), I.batch_instance(5), I.Formula(4), I.Formula(0),
              I.disjoint_union(I.small_1in3(2), I.cvc(24, 0))]:
        net = tn.Network(f)
        # "learned" runs the judge: the learned plan only when cheapest
        p = net.order("learned", seed=0, model=m)
        assert p.verify()
        rep = cost.replay(_labels(f), p.steps())
        assert rep["max_rank"] == p.stats["max_rank"]
        if _labels(f):
            assert rep["remaining"] == [[]]


def test_judge_falls_back_on_useless_weights():
    # all-zero weights score every pair alike: the learned order degenerates
    # and the judge must keep a heuristic plan and say so. (The judge's
    # search is time-budgeted, so two judge runs need not try the same
    # candidates; the comparison is with the degenerate learned order itself.)
    zero = tn.Model()
    fallbacks = 0
    for s in range(6):
        net = tn.Network(I.cvc(60, s))
        lp = net.order("learned", seed=0, model=zero)
        assert lp.verify()
        try:
            raw = net.order("learned_raw", seed=0, model=zero)
            assert lp.stats["log2_cost"] <= raw.stats["log2_cost"] + 1e-9
        except tn.TNError:
            pass  # the degenerate order exceeds the rank cap
        if lp.stats["fallback"]:
            assert lp.stats["chosen"] != "learned"
        fallbacks += lp.stats["fallback"]
    assert fallbacks >= 5


def test_learned_without_model_is_the_judge():
    net = tn.Network(I.cvc(60, 1))
    lp = net.order("learned", seed=0)
    assert lp.stats["fallback"] and lp.stats["chosen"] in ("greedy", "partition", "community")


def test_learned_hands_costly_plans_to_the_judge():
    # held-out instance 40: the learned order exceeds the rank cap and
    # greedy's plan is predicted at seconds; the judge, given it as the
    # incumbent, must return a plan no costlier and flag the fallback
    model = tn.Model.load_file(MODEL)
    net = tn.Network(I.learned_instance(40, "heldout"))
    g = net.order("greedy")
    assert 2 ** g.stats["log2_cost"] > 50000.0
    lp = net.order("learned", seed=40, model=model)
    assert lp.verify()
    assert lp.stats["log2_cost"] <= g.stats["log2_cost"] + 1e-9
    assert 2 ** lp.stats["log2_cost"] < 2 ** g.stats["log2_cost"] / 10
    assert lp.stats["fallback"] == (lp.stats["chosen"] != "learned")
    # a cheap instance stays with the learned or greedy plan (no search)
    small = tn.Network(I.learned_instance(1, "heldout"))
    sp = small.order("learned", seed=1, model=model)
    if 2 ** sp.stats["log2_cost"] <= 50000.0:
        assert sp.stats["chosen"] in ("learned", "greedy")
