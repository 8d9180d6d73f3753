"""Fig. 4(c) of the paper as a host-only series: the largest tensor rank met
along the recursive-bisection (tensor-METIS) contraction sequence -- the
largest degree of the contracted graph, which sets the cost (Sec. 3.1.1,
Corollary 2) -- averaged over random cubic graphs, against the number of
vertices |V|, for unrestricted and for planar cubic graphs, on the
#Cubic-Vertex-Cover networks of Sec. 3.2.

    python -m paper_1805_00475_amd.fig4c [--seeds 20] [--sizes 32,56,...,200]

Unrestricted graphs come from the configuration model, planar ones are duals
of random triangulations (``instances.planar_cubic_graph``). Prints a
markdown table: |V|, mean and spread of the largest rank for each family.
Planar cubic graphs have separators of O(sqrt |V|) (Sec. 3.1), so their
largest rank grows like sqrt |V|; random cubic graphs are expanders and grow
linearly.
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def series(sizes, seeds, order="partition"):
    import instances as I
    from paper_1805_00475_amd import tn
    rows = []
    for n in sizes:
        out = {}
        for fam in ("unrestricted", "planar"):
            ranks = []
            for s in range(seeds):
                rng = I.Rng(I.instance_seed(7 if fam == "unrestricted" else 8, (n << 20) | s))
                edges = I.cubic_graph(n, rng) if fam == "unrestricted" else I.planar_cubic_graph(n, rng)
                net = tn.Network(I.vertex_cover_formula(edges, n))
                try:
                    ranks.append(net.order(order, seed=s).stats["max_rank"])
                except tn.TNError:
                    ranks.append(None)  # beyond the rank cap
            ok = [r for r in ranks if r is not None]
            out[fam] = (sum(ok) / len(ok) if ok else None, min(ok) if ok else None, max(ok) if ok else None,
                        len(ranks) - len(ok))
        rows.append((n, out))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=20)
    ap.add_argument("--sizes", default="32,56,80,104,128,152,176,200")
    ap.add_argument("--order", default="partition")
    args = ap.parse_args()
    rows = series([int(x) for x in args.sizes.split(",")], args.seeds, args.order)
    print(f"| abs(V) | unrestricted: mean largest rank (min-max) | planar: mean largest rank (min-max) |")
    print("|---|---|---|")
    for n, out in rows:
        cells = []
        for fam in ("unrestricted", "planar"):
            mean, lo, hi, over = out[fam]
            cells.append(f"{mean:.2f} ({lo}-{hi})" + (f", {over} over the cap" if over else "") if mean else "-")
        print(f"| {n} | {cells[0]} | {cells[1]} |")


if __name__ == "__main__":
    main()
