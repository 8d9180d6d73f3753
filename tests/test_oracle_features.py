"""Pins of the learned order's pair features and imitation traces
(``oracle.mlp.pair_features``, ``oracle.mlp.trace``) on networks worked out
by hand, and planted mistakes that those pins must catch.

Hand-worked network (five tensors, six bonds, every bond joins two tensors):

    T0 {1, 2}   T1 {2, 3, 4}   T2 {3, 5}   T3 {4, 5, 6}   T4 {1, 6}

Neighbour sets (other tensors sharing a bond): N0 = {1, 4}, N1 = {0, 2, 3},
N2 = {1, 3}, N3 = {1, 2, 4}, N4 = {0, 3}. A pair's features, larger rank
first (ties: more neighbours first), are
    rA/32, rB/32, s/32, rC/32, (rC - rA)/8, dA/16, dB/16, c/8, (rA + rB - s)/48, [s == rB]
with s shared bonds, rC = rA + rB - 2s, c common neighbours. Every expected
row below was derived on paper from the bond lists above, not computed.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import mlp

RING = [{1, 2}, {2, 3, 4}, {3, 5}, {4, 5, 6}, {1, 6}]


def _live(sets):
    return {i: frozenset(s) for i, s in enumerate(sets)}


def _row(*vals):
    return np.array([float(Fr(v)) for v in vals])


# state 0 of the ring: (pair) -> features, worked by hand
STATE0 = {
    # T1 (rank 3, 3 nbrs) before T0 (rank 2); bond 2; rC = 3; common: {2,3} & {4} = {}
    (0, 1): _row("3/32", "2/32", "1/32", "3/32", "0", "3/16", "2/16", "0", "4/48", "0"),
    # equal ranks and neighbour counts: order kept; bond 1; rC = 2; common {1} & {3} = {}
    (0, 4): _row("2/32", "2/32", "1/32", "2/32", "0", "2/16", "2/16", "0", "3/48", "0"),
    # bond 3; common {0,3} & {3} = {3}
    (1, 2): _row("3/32", "2/32", "1/32", "3/32", "0", "3/16", "2/16", "1/8", "4/48", "0"),
    # bond 4; rC = 4 (rank grows by one); common {0,2} & {2,4} = {2}
    (1, 3): _row("3/32", "3/32", "1/32", "4/32", "1/8", "3/16", "3/16", "1/8", "5/48", "0"),
    # T3 first; bond 5; common {1,4} & {1} = {1}
    (2, 3): _row("3/32", "2/32", "1/32", "3/32", "0", "3/16", "2/16", "1/8", "4/48", "0"),
    # bond 6; common {1,2} & {0} = {}
    (3, 4): _row("3/32", "2/32", "1/32", "3/32", "0", "3/16", "2/16", "0", "4/48", "0"),
}

# after merging T1 and T3 into T5 = {2, 3, 5, 6}: N0 = {4, 5}, N2 = {5},
# N4 = {0, 5}, N5 = {0, 2, 4}
STATE1_SETS = {0: frozenset({1, 2}), 2: frozenset({3, 5}), 4: frozenset({1, 6}), 5: frozenset({2, 3, 5, 6})}
STATE1 = {
    # T5 first; bonds 3 and 5 (s = 2 = rB: T2 is absorbed whole); rC = 2
    (2, 5): _row("4/32", "2/32", "2/32", "2/32", "-2/8", "3/16", "1/16", "0", "4/48", "1"),
    # common {2,4} & {4} = {4}
    (0, 5): _row("4/32", "2/32", "1/32", "4/32", "0", "3/16", "2/16", "1/8", "5/48", "0"),
    # common {5} & {5} = {5}
    (0, 4): _row("2/32", "2/32", "1/32", "2/32", "0", "2/16", "2/16", "1/8", "3/48", "0"),
    # common {0,2} & {0} = {0}
    (4, 5): _row("4/32", "2/32", "1/32", "4/32", "0", "3/16", "2/16", "1/8", "5/48", "0"),
}

# merges of the ring: T1+T3 -> 5, T2+T5 -> 6 {2, 6}, T0+T4 -> 7 {2, 6}, T6+T7 -> 8 {}
RING_MERGES = [(1, 3), (2, 5), (0, 4), (6, 7)]
SAME = _row("2/32", "2/32", "1/32", "2/32", "0", "2/16", "2/16", "1/8", "3/48", "0")
RING_TRACE = [
    # before merge 0: the teacher merges (1,3) now and (0,4) later, both alive
    {(0, 1): (STATE0[(0, 1)], 0), (0, 4): (STATE0[(0, 4)], 1), (1, 2): (STATE0[(1, 2)], 0),
     (1, 3): (STATE0[(1, 3)], 1), (2, 3): (STATE0[(2, 3)], 0), (3, 4): (STATE0[(3, 4)], 0)},
    {(0, 4): (STATE1[(0, 4)], 1), (0, 5): (STATE1[(0, 5)], 0), (2, 5): (STATE1[(2, 5)], 1),
     (4, 5): (STATE1[(4, 5)], 0)},
    # live T0 {1,2}, T4 {1,6}, T6 {2,6}: a triangle, every pair alike
    {(0, 4): (SAME, 1), (0, 6): (SAME, 0), (4, 6): (SAME, 0)},
    # T6 and T7 share both bonds: rC = 0, rank drop 2, absorbed whole
    {(6, 7): (_row("2/32", "2/32", "2/32", "0", "-2/8", "1/16", "1/16", "0", "2/48", "1"), 1)},
]

# two disconnected bonds; the last merge joins two scalars that share nothing
PAIRS = [{1}, {1}, {2}, {2}]
PAIRS_MERGES = [(0, 1), (2, 3), (4, 5)]
ONE = _row("1/32", "1/32", "1/32", "0", "-1/8", "1/16", "1/16", "0", "1/48", "1")
PAIRS_TRACE = [
    {(0, 1): (ONE, 1), (2, 3): (ONE, 1)},
    {(2, 3): (ONE, 1)},
    # not connected: appended as the teacher's pair, all-zero but [s == rB] = [0 == 0]
    {(4, 5): (_row(0, 0, 0, 0, 0, 0, 0, 0, 0, 1), 1)},
]


def _features_pinned():
    live = _live(RING)
    for (u, v), want in STATE0.items():
        for a, b in ((u, v), (v, u)):  # argument order must not matter
            if not np.allclose(mlp.pair_features(live, a, b), want, rtol=0, atol=1e-15):
                return False
    for (u, v), want in STATE1.items():
        if not np.allclose(mlp.pair_features(STATE1_SETS, u, v), want, rtol=0, atol=1e-15):
            return False
    return True


def _trace_pinned():
    for sets, merges, expected in ((RING, RING_MERGES, RING_TRACE), (PAIRS, PAIRS_MERGES, PAIRS_TRACE)):
        groups = mlp.trace(sets, merges)
        if len(groups) != len(expected):
            return False
        for rows, want in zip(groups, expected):
            got = {pair: (f, lab) for pair, f, lab in rows}
            if set(got) != set(want):
                return False
            for pair, (f, lab) in want.items():
                if got[pair][1] != lab or not np.allclose(got[pair][0], f, rtol=0, atol=1e-15):
                    return False
    return True


def test_pair_features_hand_worked():
    assert _features_pinned()


def test_trace_hand_worked():
    assert _trace_pinned()


# ------------------------------------------------------------ planted mistakes
def _swap_rule_reversed(live, u, v):
    # smaller tensor first: the A and B roles of every rank-dependent feature traded
    f = _ORIG(live, u, v).copy()
    if f[0] != f[1]:
        f[0], f[1] = f[1], f[0]
        f[5], f[6] = f[6], f[5]
        f[4] = (f[3] - f[0]) * 32 / 8
        f[9] = 1.0 if f[2] == f[1] else 0.0
    return f


def _mutant(kind):
    def bad(live, u, v):
        f = _ORIG(live, u, v).copy()
        if kind == "rc_drop_factor":      # rC = rA + rB - s
            f[3] = f[0] + f[1] - f[2]
        elif kind == "no_common":         # common neighbours never counted
            f[7] = 0.0
        elif kind == "degree_counts_pair":  # neighbour count excludes nothing
            f[5] += 1 / 16
        elif kind == "absorb_flag_vs_rA":  # [s == rA]
            f[9] = 1.0 if f[2] == f[0] else 0.0
        elif kind == "macs_norm":          # (rA + rB - s)/32
            f[8] = f[8] * 48 / 32
        return f
    return bad


_ORIG = mlp.pair_features


@pytest.mark.parametrize("kind", ["rc_drop_factor", "no_common", "degree_counts_pair", "absorb_flag_vs_rA",
                                  "macs_norm"])
def test_feature_mistake_caught(monkeypatch, kind):
    monkeypatch.setattr(mlp, "pair_features", _mutant(kind))
    assert not _features_pinned()
    assert not _trace_pinned()


def test_order_rule_mistake_caught(monkeypatch):
    monkeypatch.setattr(mlp, "pair_features", _swap_rule_reversed)
    assert not _features_pinned()


def test_trace_labels_only_current_merge_caught(monkeypatch):
    # a trace that marks only the teacher's next merge as positive
    orig = mlp.trace

    def bad(label_sets, merges):
        groups = orig(label_sets, merges)
        out = []
        for (a, b), rows in zip(merges, groups):
            key = (min(a, b), max(a, b))
            out.append([(p, f, 1 if p == key else 0) for p, f, _ in rows])
        return out
    monkeypatch.setattr(mlp, "trace", bad)
    assert not _trace_pinned()


def test_trace_dropping_unconnected_teacher_pair_caught(monkeypatch):
    orig = mlp.trace

    def bad(label_sets, merges):
        groups = orig(label_sets, merges)
        live = {i: frozenset(s) for i, s in enumerate(label_sets)}
        nid = len(label_sets)
        out = []
        for (a, b), rows in zip(merges, groups):
            out.append([r for r in rows if live[r[0][0]] & live[r[0][1]]])
            live[nid] = live.pop(a) ^ live.pop(b)
            nid += 1
        return out
    monkeypatch.setattr(mlp, "trace", bad)
    assert not _trace_pinned()
