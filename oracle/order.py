"""An oracle-side contraction order by recursive bisection (the paper's
tensor-METIS idea, Sec. 3.1.1 and Corollary 1), for running the pairwise
contractor O-B on networks too large for its greedy order.

Test infrastructure only. The order is data, not arithmetic: any order that
merges every tensor exactly once gives the same count (Sec. 2.1), so this
module only decides how expensive the oracle's own contraction is. It is
written independently of the library (plain Python and numpy, its own
bisection), so no order the oracle uses comes from the GPU path.

Recursive bisection. The tensor graph has one vertex per tensor and, between
two tensors, an edge weighted by the number of bonds they share. A set of
tensors is split into two halves of equal size (within one vertex) with few
cut bonds: two tries per split, as the paper does, each a spectral start (the
sign pattern of the Fiedler vector of the weighted Laplacian, cut at its
median) or a breadth-first region grown from a random vertex, each refined by
Fiduccia-Mattheyses passes (single-vertex moves of the largest gain that keep
the balance, the best prefix of a pass kept); the lower cut wins. Splitting
recurses down to single tensors.

From hierarchy to order (Corollary 1: separators of the smallest parts are
contracted first): the parts are merged bottom-up. A part's result is the
list of tensors it reduces to, one per connected component; at every node
the children's lists are joined and, among pairs that share a bond, the pair
with the smallest result rank is merged until no two share a bond. At the
root the remaining tensors (scalars or disconnected pieces) are merged in
increasing rank.
"""
from __future__ import annotations

import random
from typing import Dict, List, Sequence, Set, Tuple

import numpy as np


def _tensor_graph(label_sets: Sequence[Set[int]]):
    owner: Dict[int, List[int]] = {}
    for t, ls in enumerate(label_sets):
        for l in ls:
            owner.setdefault(l, []).append(t)
    w: List[Dict[int, int]] = [dict() for _ in label_sets]
    for ts in owner.values():
        if len(ts) == 2 and ts[0] != ts[1]:
            a, b = ts
            w[a][b] = w[a].get(b, 0) + 1
            w[b][a] = w[b].get(a, 0) + 1
    return w


def _cut(w, side: Dict[int, int]) -> int:
    c = 0
    for u, s in side.items():
        for v, k in w[u].items():
            if v in side and side[v] != s and u < v:
                c += k
    return c


def _fm(w, nodes: List[int], side: Dict[int, int], passes: int = 8) -> Dict[int, int]:
    """Fiduccia-Mattheyses refinement: within a pass a side may hold one
    vertex more than a balanced split allows; the pass keeps its best prefix
    of moves that ends balanced (|A| and |B| within one of n/2)."""
    n = len(nodes)
    lo, hi = n // 2, (n + 1) // 2
    for _ in range(passes):
        size = [sum(1 for v in nodes if side[v] == 0), 0]
        size[1] = n - size[0]
        gain = {}
        for v in nodes:
            g = 0
            for u, k in w[v].items():
                if u in side:
                    g += k if side[u] != side[v] else -k
            gain[v] = g
        locked = set()
        moves = []
        total = best_total = 0
        best_len = 0
        for _step in range(n):
            cand = None
            for v in nodes:
                if v in locked:
                    continue
                s = side[v]
                if not (lo - 1 <= size[s] - 1 and size[1 - s] + 1 <= hi + 1):
                    continue
                if cand is None or gain[v] > gain[cand] or (gain[v] == gain[cand] and v < cand):
                    cand = v
            if cand is None:
                break
            v = cand
            s = side[v]
            total += gain[v]
            side[v] = 1 - s
            size[s] -= 1
            size[1 - s] += 1
            locked.add(v)
            moves.append(v)
            for u, k in w[v].items():
                if u in side and u not in locked:
                    gain[u] += 2 * k if side[u] == s else -2 * k
            if total > best_total and lo <= size[0] <= hi:
                best_total, best_len = total, len(moves)
        for v in moves[best_len:]:
            side[v] = 1 - side[v]
        if best_total <= 0:
            break
    return side


def _spectral_start(w, nodes: List[int]) -> Dict[int, int]:
    idx = {v: i for i, v in enumerate(nodes)}
    n = len(nodes)
    L = np.zeros((n, n))
    for v in nodes:
        for u, k in w[v].items():
            if u in idx:
                L[idx[v], idx[u]] -= k
                L[idx[v], idx[v]] += k
    _, vec = np.linalg.eigh(L)
    f = vec[:, 1] if n > 1 else vec[:, 0]
    order = sorted(range(n), key=lambda i: (f[i], i))
    side = {}
    for r, i in enumerate(order):
        side[nodes[i]] = 0 if r < n // 2 else 1
    return side


def _bfs_start(w, nodes: List[int], rng: random.Random) -> Dict[int, int]:
    inside = set(nodes)
    start = nodes[rng.randrange(len(nodes))]
    seen = [start]
    mark = {start}
    q = 0
    while len(seen) < len(nodes) // 2:
        if q == len(seen):
            nxt = min(v for v in nodes if v not in mark)  # disconnected: jump
            seen.append(nxt)
            mark.add(nxt)
            continue
        v = seen[q]
        q += 1
        for u in sorted(w[v]):
            if u in inside and u not in mark and len(seen) < len(nodes) // 2:
                seen.append(u)
                mark.add(u)
    return {v: (0 if v in mark else 1) for v in nodes}


def _components(w, nodes: List[int]) -> List[List[int]]:
    inside = set(nodes)
    seen = set()
    comps = []
    for v in nodes:
        if v in seen:
            continue
        comp = [v]
        seen.add(v)
        q = 0
        while q < len(comp):
            for u in w[comp[q]]:
                if u in inside and u not in seen:
                    seen.add(u)
                    comp.append(u)
            q += 1
        comps.append(sorted(comp))
    return comps


def _bisect(w, nodes: List[int], rng: random.Random) -> Tuple[List[int], List[int]]:
    comps = _components(w, nodes)
    if len(comps) > 1:
        # a disconnected set splits along its components (no bond is cut):
        # largest first onto the smaller side
        a: List[int] = []
        b: List[int] = []
        for c in sorted(comps, key=lambda c: (-len(c), c[0])):
            (a if len(a) <= len(b) else b).extend(c)
        return sorted(a), sorted(b)
    best = None
    starts = [_spectral_start(w, nodes), _bfs_start(w, nodes, rng)] if len(nodes) > 2 else \
        [{v: i for i, v in enumerate(nodes)}]
    if seeded_spectral_off(rng):
        starts = starts[1:] + [_bfs_start(w, nodes, rng)]
    for side in starts:
        side = _fm(w, nodes, dict(side))
        c = _cut(w, side)
        if best is None or c < best[0]:
            best = (c, side)
    side = best[1]
    return [v for v in nodes if side[v] == 0], [v for v in nodes if side[v] == 1]


def seeded_spectral_off(rng: random.Random) -> bool:
    """Tries after the first replace the spectral start by a second random
    breadth-first start (the spectral start is deterministic)."""
    return getattr(rng, "no_spectral", False)


def _absorb_small(label_sets: List[frozenset]):
    """Merge every tensor of rank <= 2 into the neighbour it shares most bonds
    with (ties: lower id); such a merge never raises a rank. Returns the merges
    and the surviving tensors as {id: labels}."""
    live: Dict[int, frozenset] = {i: s for i, s in enumerate(label_sets)}
    nid = len(label_sets)
    merges = []
    changed = True
    while changed:
        changed = False
        owner: Dict[int, List[int]] = {}
        for t, ls in live.items():
            for l in ls:
                owner.setdefault(l, []).append(t)
        for t in sorted(live):
            if t not in live or not (0 < len(live[t]) <= 2):
                continue
            share: Dict[int, int] = {}
            for l in live[t]:
                for u in owner.get(l, []):
                    if u != t and u in live:
                        share[u] = share.get(u, 0) + 1
            if not share:
                continue
            u = min(share, key=lambda x: (-share[x], x))
            live[nid] = live.pop(t) ^ live.pop(u)
            merges.append((min(t, u), max(t, u)))
            nid += 1
            changed = True
            break
    return merges, live, nid


def partition_order(label_sets: Sequence[Sequence[int]], seed: int = 0, tries: int = 1
                    ) -> List[Tuple[int, int]]:
    """Merges (i, j) of tensor ids; merge k creates id len(label_sets) + k.
    With tries > 1, the order with the fewest multiply-adds among ``tries``
    seeded runs (the first with a spectral start) is returned."""
    if tries > 1:
        best = None
        for t in range(tries):
            m = partition_order(label_sets, seed * 1000003 + t, 1) if t else partition_order(label_sets, seed, 1)
            c = _macs(label_sets, m)
            if best is None or c < best[0]:
                best = (c, m)
        return best[1]
    merges, live, next_id = _absorb_small([frozenset(ls) for ls in label_sets])
    ids = sorted(live)
    # the bisection runs on the surviving tensors, relabelled 0..k-1
    sets = [set(live[i]) for i in ids]
    w = _tensor_graph(sets)
    rng = random.Random(seed)
    if seed % 2:
        rng.no_spectral = True
    nid = [next_id]

    def merge(a: int, b: int) -> int:
        live[nid[0]] = live.pop(a) ^ live.pop(b)
        merges.append((a, b))
        nid[0] += 1
        return nid[0] - 1

    def merge(a: int, b: int) -> int:
        live[nid[0]] = live.pop(a) ^ live.pop(b)
        merges.append((a, b))
        nid[0] += 1
        return nid[0] - 1

    def join(parts: List[int], connected_only: bool) -> List[int]:
        parts = list(parts)
        while len(parts) > 1:
            best = None
            for i in range(len(parts)):
                for j in range(i + 1, len(parts)):
                    a, b = parts[i], parts[j]
                    sh = live[a] & live[b]
                    if connected_only and not sh:
                        continue
                    key = (len(live[a] ^ live[b]), min(a, b), max(a, b))
                    if best is None or key < best[0]:
                        best = (key, i, j)
            if best is None:
                break
            _, i, j = best
            c = merge(parts[i], parts[j])
            parts = [p for k, p in enumerate(parts) if k not in (i, j)] + [c]
        return parts

    def solve(nodes: List[int]) -> List[int]:
        if len(nodes) == 1:
            return [ids[nodes[0]]]
        a, b = _bisect(w, nodes, rng)
        return join(solve(a) + solve(b), True)

    if not label_sets:
        return []
    rest = solve(list(range(len(sets)))) if sets else []
    join(sorted(rest, key=lambda t: (len(live[t]), t)), False)
    return merges


def _macs(label_sets, merges) -> int:
    live = {i: frozenset(s) for i, s in enumerate(label_sets)}
    nid = len(label_sets)
    total = 0
    for a, b in merges:
        x, y = live.pop(a), live.pop(b)
        total += 1 << (len(x) + len(y) - len(x & y))
        live[nid] = x ^ y
        nid += 1
    return total


# ------------------------------------------------------------ Girvan-Newman
def _edge_betweenness(adj: Dict[int, Set[int]], nodes: List[int]) -> Dict[Tuple[int, int], float]:
    """Brandes' accumulation of shortest-path counts over every source, for
    the edges of an unweighted simple graph restricted to ``nodes``."""
    bet: Dict[Tuple[int, int], float] = {}
    for s in nodes:
        order = [s]
        sigma = {s: 1.0}
        dist = {s: 0}
        preds: Dict[int, List[int]] = {s: []}
        q = 0
        while q < len(order):
            v = order[q]
            q += 1
            for u in adj[v]:
                if u not in dist:
                    dist[u] = dist[v] + 1
                    sigma[u] = 0.0
                    preds[u] = []
                    order.append(u)
                if dist[u] == dist[v] + 1:
                    sigma[u] += sigma[v]
                    preds[u].append(v)
        delta = {v: 0.0 for v in order}
        for v in reversed(order):
            for u in preds[v]:
                c = sigma[u] / sigma[v] * (1.0 + delta[v])
                e = (min(u, v), max(u, v))
                bet[e] = bet.get(e, 0.0) + c
                delta[u] += c
    return bet


def community_order(label_sets: Sequence[Sequence[int]]) -> List[Tuple[int, int]]:
    """Order from a Girvan-Newman split tree (the paper's tensor-GN,
    Sec. 3.1.1): on the simple graph of the tensors left after absorbing
    those of rank <= 2, repeatedly delete the edge of largest betweenness
    (recomputed in the component that lost an edge; ties to the smallest
    edge); a deletion that disconnects a component splits it into two
    children. The tree is merged bottom-up like the bisection hierarchy."""
    merges, live, next_id = _absorb_small([frozenset(ls) for ls in label_sets])
    ids = sorted(live)
    k = len(ids)
    sets = [set(live[i]) for i in ids]
    w = _tensor_graph(sets)
    adj: Dict[int, Set[int]] = {v: set(w[v]) for v in range(k)}
    children: Dict[int, Tuple[int, int]] = {}
    members: Dict[int, List[int]] = {}
    # tree nodes: leaves 0..k-1 are tensors; inner nodes get ids from k up
    comp_node: Dict[int, int] = {}
    nxt = [k]

    def new_node(vs: List[int]) -> int:
        if len(vs) == 1:
            return vs[0]
        t = nxt[0]
        nxt[0] += 1
        members[t] = sorted(vs)
        return t

    roots = []
    for comp in _components(w, list(range(k))):
        r = new_node(comp)
        roots.append(r)
        for v in comp:
            comp_node[v] = r
    work = [r for r in roots if r >= k]
    while work:
        t = work.pop()
        vs = members[t]
        while True:
            bet = _edge_betweenness(adj, vs)
            e = max(bet, key=lambda x: (bet[x], -x[0], -x[1]))
            adj[e[0]].discard(e[1])
            adj[e[1]].discard(e[0])
            comps = _components({v: adj[v] for v in range(k)}, vs)
            if len(comps) > 1:
                a, b = comps[0], comps[1]
                ca, cb = new_node(a), new_node(b)
                children[t] = (ca, cb)
                work += [c for c in (ca, cb) if c >= k]
                break

    nid = [next_id]

    def merge(a: int, b: int) -> int:
        live[nid[0]] = live.pop(a) ^ live.pop(b)
        merges.append((a, b))
        nid[0] += 1
        return nid[0] - 1

    def join(parts: List[int], connected_only: bool) -> List[int]:
        parts = list(parts)
        while len(parts) > 1:
            best = None
            for i in range(len(parts)):
                for j in range(i + 1, len(parts)):
                    a, b = parts[i], parts[j]
                    if connected_only and not (live[a] & live[b]):
                        continue
                    key = (len(live[a] ^ live[b]), min(a, b), max(a, b))
                    if best is None or key < best[0]:
                        best = (key, i, j)
            if best is None:
                break
            _, i, j = best
            c = merge(parts[i], parts[j])
            parts = [p for q, p in enumerate(parts) if q not in (i, j)] + [c]
        return parts

    def solve(t: int) -> List[int]:
        if t < k:
            return [ids[t]]
        a, b = children[t]
        return join(solve(a) + solve(b), True)

    if not label_sets:
        return []
    rest = []
    for r in roots:
        rest += solve(r)
    join(sorted(rest, key=lambda t: (len(live[t]), t)), False)
    return merges


def cheapest_order(label_sets: Sequence[Sequence[int]], tries: int = 16, community: bool = True
                   ) -> Tuple[List[Tuple[int, int]], str]:
    """The order with the fewest multiply-adds among the bisection tries and
    (optionally) the Girvan-Newman order; returns (merges, which)."""
    cands = [(partition_order(label_sets, 0, tries), "partition")]
    if community:
        cands.append((community_order(label_sets), "community"))
    return min(cands, key=lambda c: _macs(label_sets, c[0]))
