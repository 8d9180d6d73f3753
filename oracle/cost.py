"""Symbolic replay of a pairwise contraction order (the "lazy" cost check of
Sec. 4: contract the graph first, track degrees, and know the cost before
touching any tensor entry).

A tensor is tracked only by its set of bond labels. Merging tensors with
label sets SA and SB shares s = |SA & SB| bonds and yields rank
|SA ^ SB| = rA + rB - 2s (Sec. 2.1). For one step:
    entries moved  = 2^rA + 2^rB + 2^rC      (read A, read B, write C)
    multiply-adds  = 2^(rA + rB - s)          (every output entry sums 2^s products)
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple


def replay(label_sets: Sequence[Sequence[int]], order: Sequence[Tuple[int, int]]):
    live: Dict[int, frozenset] = {i: frozenset(s) for i, s in enumerate(label_sets)}
    nid = len(label_sets)
    steps = []
    for i, j in order:
        a = live.pop(i)
        b = live.pop(j)
        s = len(a & b)
        c = a ^ b
        steps.append({"rA": len(a), "rB": len(b), "s": s, "rC": len(c),
                      "entries": 2 ** len(a) + 2 ** len(b) + 2 ** len(c),
                      "macs": 2 ** (len(a) + len(b) - s)})
        live[nid] = c
        nid += 1
    return {
        "steps": steps,
        "max_rank": max([max((len(s) for s in label_sets), default=0)] + [st["rC"] for st in steps]),
        "entries": sum(st["entries"] for st in steps),
        "macs": sum(st["macs"] for st in steps),
        "remaining": [sorted(v) for _, v in sorted(live.items())],
    }
