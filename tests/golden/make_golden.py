"""Writes the stored expected counts under tests/golden from the oracle only.

    python tests/golden/make_golden.py [--large]
    python tests/golden/make_golden.py --cvc200 [seeds...]

cvc200_counts.json        vertex cover of random cubic graphs, n=200: the
                          pairwise contractor O-B (exact float64 limb products
                          per 31-bit prime, CRT) along the oracle's own order
                          (oracle.order: the cheaper of its Girvan-Newman and
                          bisection orders), checked against one extra prime

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
from oracle import brute, contract, elim, order, rns, tensors  # noqa: E402


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


def count_ob(f, log=print):
    """O-B along the oracle's cheapest own order, one 31-bit prime at a time,
    with the CRT result checked modulo one more prime."""
    nets, _ = tensors.network_of_formula(f)
    labels = [ls for _, ls in nets]
    t = time.time()
    merges, which = order.cheapest_order(labels)
    mr = order_max_rank(labels, merges)
    log(f"  {f.name}: {which} order, max rank {mr} ({time.time() - t:.1f}s)")
    primes = rns.primes_for(f.n_vars)
    extra = rns.largest_primes_below(1 << 31, len(primes) + 1)[-1]
    res = []
    for p in primes + [extra]:
        t = time.time()
        res.append(contract.count_mod(f, p, merges))
        log(f"    mod {p}: {res[-1]} ({time.time() - t:.1f}s)")
    c = rns.crt(res[:-1], primes)
    assert c % extra == res[-1], "extra-prime check failed"
    return c, which, mr


def order_max_rank(labels, merges):
    return contract.max_rank_of_order(labels, merges)


def cvc200(seeds):
    path = os.path.join(HERE, "cvc200_counts.json")
    items = json.load(open(path))["items"] if os.path.exists(path) else []
    have = {it["seed"] for it in items}
    for s in seeds:
        if s in have:
            continue
        f = I.cvc(200, s)
        c, which, mr = count_ob(f)
        items.append({"n": 200, "seed": s, "count": str(c), "order": which, "max_rank": mr})
        items.sort(key=lambda it: it["seed"])
        dump("cvc200_counts.json", {
            "workload": "instances.cvc(200, seed): vertex covers of a uniform random cubic graph, n=200",
            "oracle": "oracle.contract.count_mod (O-B) per prime of oracle.rns.primes_for(200) along "
                      "oracle.order.cheapest_order, oracle.rns.crt; checked modulo one extra prime",
            "items": items})


# uniform 1-in-3 instances of the large workload (n = 150-300, alpha
# 0.62-0.70) small enough for a CPU oracle: O-B along the oracle's own order
# where that order stays at rank <= 28, O-D where its elimination width does
C3_CASES = [(200, 0.66, 0, "ob"), (200, 0.66, 1, "od"), (200, 0.66, 3, "ob"), (200, 0.70, 3, "ob"),
            (250, 0.62, 1, "ob"), (200, 0.62, 0, "ob"), (200, 0.62, 1, "ob+od"), (200, 0.62, 2, "ob+od"),
            (200, 0.62, 3, "ob"), (200, 0.62, 4, "ob"), (200, 0.62, 5, "ob"), (250, 0.62, 4, "ob")]


def c3():
    path = os.path.join(HERE, "c3_1in3_counts.json")
    items = json.load(open(path))["items"] if os.path.exists(path) else []
    have = {(it["n"], it["alpha"], it["seed"]) for it in items}
    for n, a, s, how in C3_CASES:
        if (n, a, s) in have:
            continue
        f = I.large_1in3(n, a, s)
        t = time.time()
        if how.startswith("ob"):
            c, which, mr = count_ob(f)
            it = {"n": n, "alpha": a, "seed": s, "count": str(c), "oracle": "O-B", "order": which, "max_rank": mr}
            if how == "ob+od":
                assert elim.count_rns(f) == c, "O-B and O-D disagree"
                it["oracle"] = "O-B, O-D"
        else:
            c = elim.count_rns(f)
            it = {"n": n, "alpha": a, "seed": s, "count": str(c), "oracle": "O-D", "width": elim.width(f)}
        print(f"  1in3 n={n} a={a} s={s}: {c} ({time.time() - t:.1f}s)", flush=True)
        items.append(it)
        items.sort(key=lambda x: (x["n"], x["alpha"], x["seed"]))
        dump("c3_1in3_counts.json", {
            "workload": "instances.large_1in3(n, alpha, seed): monotone 1-in-3, clauses of 3 distinct uniform "
                        "variables, m = round(alpha n)",
            "oracle": "O-B: oracle.contract.count_mod per 31-bit prime along oracle.order.cheapest_order + "
                      "oracle.rns.crt, checked modulo one extra prime; O-D: oracle.elim.count_rns",
            "items": items})


# the paper's own 1-in-3 family (Sec. 3.2): cubic graphs on nv vertices, one
# variable per edge (N = 3 nv / 2), one exactly-one clause per vertex; the
# solutions are the perfect matchings. O-B along the oracle's own order, and
# O-D as well where its elimination width is small.
F1_CASES = [(60, 0, "ob+od"), (60, 1, "ob+od"), (60, 2, "ob+od"), (100, 0, "ob"), (100, 1, "ob"), (100, 2, "ob"),
            (140, 0, "ob"), (140, 1, "ob"), (140, 2, "ob"), (200, 1, "ob")]


def f1():
    path = os.path.join(HERE, "cubic_1in3_counts.json")
    items = json.load(open(path))["items"] if os.path.exists(path) else []
    have = {(it["n_vertices"], it["seed"]) for it in items}
    for nv, s, how in F1_CASES:
        if (nv, s) in have:
            continue
        f = I.cubic_1in3(nv, s)
        t = time.time()
        c, which, mr = count_ob(f)
        it = {"n_vertices": nv, "n_vars": f.n_vars, "seed": s, "count": str(c), "oracle": "O-B", "order": which,
              "max_rank": mr}
        if how == "ob+od":
            assert elim.count_rns(f) == c, "O-B and O-D disagree"
            it["oracle"] = "O-B, O-D"
        print(f"  cubic 1-in-3 nv={nv} s={s}: {c} ({time.time() - t:.1f}s)", flush=True)
        items.append(it)
        items.sort(key=lambda x: (x["n_vertices"], x["seed"]))
        dump("cubic_1in3_counts.json", {
            "workload": "instances.cubic_1in3(n_vertices, seed): the paper's 1-in-3 family, one variable per edge "
                        "of a uniform random cubic graph, one exactly-one clause per vertex (perfect matchings)",
            "oracle": "O-B: oracle.contract.count_mod per 31-bit prime along oracle.order.cheapest_order + "
                      "oracle.rns.crt, checked modulo one extra prime; O-D: oracle.elim.count_rns",
            "items": items})


def batch256():
    """The first 256 instances of the mixed batch: O-A for n <= 32, else O-D."""
    items = []
    for i in range(256):
        f = I.batch_instance(i)
        c = brute.count_c(f) if f.n_vars <= 32 else elim.count_rns(f)
        items.append({"index": i, "n_vars": f.n_vars, "count": str(c),
                      "oracle": "O-A" if f.n_vars <= 32 else "O-D"})
        if i % 32 == 31:
            print(f"  batch {i + 1}/256", flush=True)
    dump("batch256_counts.json", {
        "workload": "instances.batch_instance(i), master seed 0, i < 256 (even: monotone 1-in-3 n~U[30,120], "
                    "m=round(0.66n); odd: vertex cover of a random cubic graph, n~U[30,120] rounded up to even)",
        "oracle": "oracle.brute.count_c (O-A) for n <= 32, else oracle.elim.count_rns (O-D)", "items": items})


if __name__ == "__main__":
    if "--f1" in sys.argv:
        f1()
    elif "--batch256" in sys.argv:
        batch256()
    elif "--c3" in sys.argv:
        c3()
    elif "--cvc200" in sys.argv:
        cvc200([int(x) for x in sys.argv[sys.argv.index("--cvc200") + 1:]] or [0, 1])
    else:
        main(large="--large" in sys.argv)
