"""Writes the stored expected counts under tests/golden from the oracle only.

    python tests/golden/make_golden.py [--large]

small_1in3_counts.json    monotone 1-in-3, n=20, m=14, seeds 0..999 (O-A brute force)
batch_small_counts.json   the first instances of the mixed batch with n <= 30 (O-A)
batch_counts.json         mixed batch instances 0..47 (O-A for n <= 30, else O-D)
cvc_counts.json           vertex cover of random cubic graphs, n=60 (O-A is out of
                          reach; bucket elimination O-D, cross-checked by the
                          pairwise contractor O-B) and n=120 (O-D); with --large
                          also n=200 seeds 0..1 (O-D)
large_1in3_counts.json    1-in-3 n=150 alpha=0.66 seeds 0..2 (O-D); --large adds n=200
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import instances as I  # noqa: E402
from oracle import brute, contract, elim  # noqa: E402


def dump(name, obj):
    with open(os.path.join(HERE, name), "w") as fh:
        json.dump(obj, fh, indent=1)
    print("wrote", name)


def main(large=False):
    t = time.time()
    counts = [brute.count_c(I.small_1in3(i)) for i in range(1000)]
    dump("small_1in3_counts.json", {
        "workload": "monotone 1-in-3, n=20, m=14, clause = 3 distinct uniform variables; instances.small_1in3(i)",
        "oracle": "oracle.brute.count_c (O-A)", "counts": counts})
    print(f"  {time.time() - t:.1f}s")

    items = []
    i = 0
    while len(items) < 24:
        f = I.batch_instance(i)
        if f.n_vars <= 32:
            items.append({"index": i, "n_vars": f.n_vars, "count": brute.count_c(f)})
        i += 1
    dump("batch_small_counts.json", {
        "workload": "instances.batch_instance(i), master seed 0, the first 24 with n <= 32",
        "oracle": "oracle.brute.count_c (O-A)", "items": items})

    bat = []
    for i in range(48):
        f = I.batch_instance(i)
        t = time.time()
        c = brute.count_c(f) if f.n_vars <= 30 else elim.count_rns(f)
        bat.append({"index": i, "n_vars": f.n_vars, "count": str(c)})
        print(f"  batch {i} n={f.n_vars}: {c} ({time.time() - t:.1f}s)")
    dump("batch_counts.json", {
        "workload": "instances.batch_instance(i), master seed 0, i < 48",
        "oracle": "oracle.brute.count_c (O-A) for n <= 30, else oracle.elim.count_rns (O-D)", "items": bat})

    cvc = []
    for n, seeds in ((60, range(10)), (120, range(6))) + (((200, range(2)),) if large else ()):
        for s in seeds:
            f = I.cvc(n, s)
            t = time.time()
            c = elim.count_rns(f)
            if n == 60:
                assert contract.count_rns(f) == c
            cvc.append({"n": n, "seed": s, "count": str(c), "width": elim.width(f)})
            print(f"  cvc n={n} s={s}: {c} ({time.time() - t:.1f}s)")
    dump("cvc_counts.json", {
        "workload": "instances.cvc(n, seed): vertex covers of a uniform random cubic graph",
        "oracle": "oracle.elim.count_rns (O-D, bucket elimination); n=60 also oracle.contract.count_rns (O-B)",
        "items": cvc})

    l13 = []
    for n, seeds in ((150, range(3)),) + (((200, range(2)),) if large else ()):
        for s in seeds:
            f = I.large_1in3(n, 0.66, s)
            t = time.time()
            c = elim.count_rns(f)
            l13.append({"n": n, "alpha": 0.66, "seed": s, "count": str(c), "width": elim.width(f)})
            print(f"  1in3 n={n} s={s}: {c} ({time.time() - t:.1f}s)")
    dump("large_1in3_counts.json", {
        "workload": "instances.large_1in3(n, alpha, seed): monotone 1-in-3 with uniform clauses",
        "oracle": "oracle.elim.count_rns (O-D)", "items": l13})


if __name__ == "__main__":
    main(large="--large" in sys.argv)
