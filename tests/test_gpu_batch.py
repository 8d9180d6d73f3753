"""Batched counting (waves of persistent launches captured in a hipGraph)
against the oracle's counts of the mixed batch, with every execution mode
(graph, direct launches, timing) and forced sub-batching."""
import json
import os

import pytest

import instances as I
from paper_1805_00475_amd import tn

GOLD = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _gold():
    with open(os.path.join(GOLD, "batch_counts.json")) as fh:
        return {it["index"]: int(it["count"]) for it in json.load(fh)["items"]}


def _run(fs, order, flags=0, ws_bytes=8 << 30):
    import torch
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = tn.count_batch(fs, order, seed=0, flags=flags, workspace_bytes_=ws_bytes)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("order", ["greedy", "best"])
def test_batch_matches_oracle(order):
    g = _gold()
    fs = [I.batch_instance(i) for i in sorted(g)]
    _say(f"batch of {len(fs)} mixed instances, {order}, hipGraph")
    got = _run(fs, order)
    assert got == [g[i] for i in sorted(g)]


def test_batch_modes_agree():
    g = _gold()
    fs = [I.batch_instance(i) for i in sorted(g)][:24]
    want = [g[i] for i in sorted(g)][:24]
    for flags, name in ((tn.FLAG_NO_GRAPH, "direct"), (tn.FLAG_TIMING, "timing"),
                        (tn.FLAG_GENERIC_ONLY | tn.FLAG_NO_GRAPH, "generic")):
        _say(f"batch mode {name}")
        assert _run(fs, "best", flags) == want


def test_batch_sub_batches():
    # a workspace of 48 MiB forces many sub-batches and single runs
    g = _gold()
    fs = [I.batch_instance(i) for i in sorted(g)]
    _say("batch with a 48 MiB workspace")
    assert _run(fs, "best", 0, ws_bytes=48 << 20) == [g[i] for i in sorted(g)]


def test_batch_degenerate_members():
    fs = [I.Formula(0), I.Formula(7), I.Formula(3, [(I.OR, [])]), I.vertex_cover_formula(I.prism_graph(100)),
          I.small_1in3(3), I.Formula(70, [(I.OR, [1, 2])])]
    from oracle import brute, closed
    want = [1, 128, 0, closed.prism_vertex_covers(100), brute.count(I.small_1in3(3)), 3 * 2 ** 68]
    _say("batch with degenerate members")
    assert _run(fs, "best") == want


def test_batch_matches_single_counts_large():
    # n = 120 instances of both families: batch path == single-instance path,
    # and the CVC ones == the oracle's stored counts
    with open(os.path.join(GOLD, "cvc_counts.json")) as fh:
        cvc = [it for it in json.load(fh)["items"] if it["n"] == 120]
    fs = [I.cvc(120, it["seed"]) for it in cvc]
    _say("batch of n=120 cubic vertex cover")
    assert _run(fs, "best") == [int(it["count"]) for it in cvc]


def test_batch_4096_first_256_match_oracle():
    # the benchmark's full mixed batch of 4096 instances, greedy order, in one
    # call; the first 256 counts against the oracle (O-A for n <= 32, else
    # O-D), the rest checked for repeatability across two calls
    with open(os.path.join(GOLD, "batch256_counts.json")) as fh:
        want = [int(it["count"]) for it in json.load(fh)["items"]]
    fs = [I.batch_instance(i) for i in range(4096)]
    _say("batch of 4096 mixed instances, greedy, hipGraph")
    got = _run(fs, "greedy", ws_bytes=64 << 30)
    assert got[:256] == want
    _say("batch of 4096 again, direct launches")
    assert _run(fs, "greedy", flags=tn.FLAG_NO_GRAPH, ws_bytes=64 << 30) == got
