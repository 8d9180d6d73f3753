"""Benchmark: exact counts per second of #Cubic-Vertex-Cover on random cubic
graphs (Sec. 3.2 workload; configuration model, n = 200 vertices by
default), counted by tensor-network contraction on one MI355X.

A step is one pass of the whole path over one batch of formulas: build the
network, order it on the host, contract on the GPU, recombine by CRT. The
timed region starts with the formulas in host memory (the path's input);
every count is exact.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 200] [--batch B]
                    [--order best] [--no-cpu-baseline]

Prints one JSON line. ``roofline`` reports the dominant kernel class measured
with hipEvents around every launch of an extra, identical pass;
``cpu_baseline`` times the CPU oracle on a bounded sample of the workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the matrix-core kernels (small-modulus residues)
# from rocprofv3 byte counters (FETCH_SIZE and WRITE_SIZE runs of this
# benchmark, scaled by a plain copy of known size); used only while the kernel
# source is the one measured
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_mfma8_cvc200_batch16_traffic.txt")
INT8_PEAK_TOPS = 5000.0   # dense int8 MFMA, MI355X
# int8 products per multiply-add modulo one modulus: 4 digit pairs for the
# 16-bit primes, 1 for small moduli (centred int8 residues); an int8 op is a
# multiply or an add, 2 per product
INT8_PRODUCTS_PER_MODMAC = {"wide": 4, "small": 1}


def measured_traffic():
    """Counter-derived bytes per k_mfma launch, or None when the kernel
    source changed since the counters were taken (or no record exists)."""
    import hashlib
    try:
        rec = {}
        for line in open(TRAFFIC_FILE):
            if line.strip() and not line.startswith("#"):
                key, _, val = line.partition(":")
                rec[key.strip()] = val.strip()
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def roofline_of(name, d, mode="small"):
    """Achieved vs peak for one kernel class from its hipEvent total.

    Matrix-core GEMM (mfma): algorithmic multiply-adds modulo each modulus,
    each costing INT8_PRODUCTS_PER_MODMAC[mode] int8 products (2 int8 ops
    apiece), against the dense int8 MFMA peak. Every other class: algorithmic
    bytes (entries of A and B read, C written) against the HBM peak."""
    sec = d["ms"] * 1e-3
    per = {"kernel_class": name, "launches": d["launches"],
           "avg_launch_us": round(1e6 * sec / max(1, d["launches"]), 3)}
    if name == "mfma":
        tops = d["macs"] * 2 * INT8_PRODUCTS_PER_MODMAC[mode] / sec / 1e12 if sec > 0 else 0.0
        per.update({"bound": "mfma", "achieved": round(tops, 2), "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                    "frac": round(tops / INT8_PEAK_TOPS, 4),
                    "traffic": measured_traffic() if mode == "small" else None,
                    "algorithmic_modmacs_per_launch": d["macs"] / max(1, d["launches"]),
                    "achieved_modmacs_per_s": d["macs"] / sec if sec > 0 else 0.0})
    else:
        gbs = d["bytes"] / sec / 1e9 if sec > 0 else 0.0
        per.update({"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                    "algorithmic_bytes_per_launch": d["bytes"] / max(1, d["launches"])})
    return per


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["cvc", "batch"], default="cvc",
                    help="cvc: vertex cover of random cubic graphs (n vertices); batch: the mixed batch "
                         "of 1-in-3 and cubic vertex cover with n in [30, 120]")
    ap.add_argument("--n", type=int, default=200)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--order", default="best")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned vs greedy comparison")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device (a plain copy kernel of known size, used to scale "
                         "hardware byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--single", action="store_true", help="count one formula at a time instead of the batch API")
    ap.add_argument("--wide-rns", action="store_true",
                    help="residues modulo 16-bit primes even where small int8 moduli suffice")
    return ap.parse_args()


def cpu_baseline(formula, plan_steps, budget_s):
    """Oracle O-B (numpy pairwise contraction) on one prime of one instance,
    following the same contraction order, stopped after ``budget_s``; the
    instance time is extrapolated linearly in multiply-adds done and in the
    oracle's own number of primes (31-bit ones)."""
    import numpy as np
    from oracle import contract, cost, rns, tensors
    n_primes = rns.n_primes_for(formula.n_vars)
    nets, _ = tensors.network_of_formula(formula)
    rep = cost.replay([ls for _, ls in nets], plan_steps)
    macs = [s["macs"] for s in rep["steps"]]
    total = float(sum(macs))
    p = rns.primes_for(formula.n_vars)[0]
    work = {i: (np.asarray(t, dtype=np.int64) % p, ls) for i, (t, ls) in enumerate(nets)}
    nid = len(nets)
    done = 0.0
    t0 = time.process_time()
    w0 = time.time()
    k = 0
    for k, (a, b) in enumerate(plan_steps):
        work[nid] = contract.contract_pair(work.pop(a), work.pop(b), p)
        nid += 1
        done += macs[k]
        if time.time() - w0 > budget_s:
            break
    el = time.time() - w0
    frac = done / total
    inst_s = el / max(frac, 1e-12) * n_primes
    return {"value": 1.0 / inst_s, "unit": "counts/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle O-B (numpy pairwise contraction, exact int64 limbs) on {formula.name}, "
                       f"prime 1 of {n_primes}, first {k + 1} of {len(plan_steps)} steps of the same order "
                       f"= {100 * frac:.2f}% of its multiply-adds in {el:.1f}s wall "
                       f"({time.process_time() - t0:.1f}s CPU); instance time extrapolated linearly in "
                       f"multiply-adds and primes"),
            "extrapolated_instance_s": inst_s}


LEARNED_HELDOUT = [1, 4, 6, 9, 12, 15, 16, 18, 22, 23]


def learned_vs_greedy(tn, I, ws, log):
    """Order + contraction wall time of greedy, the learned scorer alone and
    the judged learned order on held-out 1-in-3 instances (n in [100, 180],
    alpha = 0.66) where greedy stays within the rank cap."""
    import torch
    model_path = os.path.join(ROOT, "paper_1805_00475_amd", "models", "order_mlp.npy")
    if not os.path.exists(model_path):
        return None
    model = tn.Model.load_file(model_path)
    res = {}
    counts = {}
    for kind in ("greedy", "learned_raw", "learned"):
        order_s = contract_s = 0.0
        cs = []
        for i in LEARNED_HELDOUT:
            f = I.learned_instance(i, "heldout")
            net = tn.Network(f)
            t0 = time.perf_counter()
            plan = net.order(kind, seed=i, model=model if "learned" in kind else None)
            t1 = time.perf_counter()
            tn.count_plan(net, plan, workspace=ws)  # warm
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            cs.append(tn.count_plan(net, plan, workspace=ws))
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            order_s += t1 - t0
            contract_s += t3 - t2
        counts[kind] = cs
        res[kind] = {"order_ms": round(1000 * order_s, 3), "contract_ms": round(1000 * contract_s, 3),
                     "total_ms": round(1000 * (order_s + contract_s), 3)}
    if not (counts["greedy"] == counts["learned_raw"] == counts["learned"]):
        raise SystemExit("learned and greedy orders disagree on a count")
    res["instances"] = f"held-out learned_instance {LEARNED_HELDOUT}"
    res["learned_over_greedy_speedup"] = round(res["greedy"]["total_ms"] / res["learned_raw"]["total_ms"], 3)
    log("learned vs greedy done")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(multi-GPU sharding of the path is described in DESIGN.md, not implemented)"}))
        sys.exit(2)
    import torch
    import instances as I
    from paper_1805_00475_amd import tn
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    base_flags = tn.FLAG_WIDE_RNS if args.wide_rns else 0
    mode = "wide" if args.wide_rns else "small"
    res_desc = ("residues mod 16-bit primes (the fewest whose product exceeds 2^(n+1))" if args.wide_rns else
                "centred int8 residues mod pairwise coprime moduli <= 255 (the fewest whose product exceeds "
                "2^(n+1))")
    if args.workload == "cvc":
        formulas = [I.cvc(args.n, s) for s in range(args.batch)]
        mods = tn.moduli(tn.Network(formulas[0]).order("community"), flags=base_flags)
        k_primes = len(mods)
        workload = (f"#Cubic-Vertex-Cover, uniform random cubic graphs n={args.n} (configuration model), "
                    f"batch of {args.batch} seeds, {args.order} order, {k_primes} moduli + CRT; {res_desc}")
    else:
        formulas = [I.batch_instance(i) for i in range(args.batch)]
        k_primes = None
        workload = (f"mixed batch of {args.batch}: even index monotone 1-in-3 n~U[30,120] m=round(0.66n), "
                    f"odd index cubic vertex cover n~U[30,120] (even); {args.order} order; u64 for n<=63 else "
                    f"{res_desc}")
    ws = tn.default_workspace()
    ws.get(64 << 30)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def one_pass(flags=0):
        flags |= base_flags
        if args.single:
            return [tn.count(f, args.order, seed=i, flags=flags, workspace=ws) for i, f in enumerate(formulas)]
        return tn.count_batch(formulas, args.order, seed=0, flags=flags, workspace=ws, with_stats=False)

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        ref = one_pass()
        log("warmup pass done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        got = one_pass()
        log(f"timed step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if args.warmup and got != ref:
        raise SystemExit("counts changed between passes")
    ms_per_step = 1000.0 * (t1 - t0) / args.steps
    value = args.batch * args.steps / (t1 - t0)

    # roofline: one more identical pass with hipEvents around every launch
    # (on the library's stream, which is torch's current stream)
    one_pass(tn.FLAG_TIMING)
    prof = tn.profile()
    log("timing pass done")
    dom = max(prof, key=lambda k: prof[k]["ms"])
    roofline = roofline_of(dom, prof[dom], mode)
    per_class = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                     "algorithmic_GBps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None,
                     "avg_launch_us": round(1000.0 * v["ms"] / v["launches"], 3)}
                 for k, v in prof.items() if v["launches"]}

    lvg = learned_vs_greedy(tn, I, ws, log) if not args.no_learned else None
    plans = [tn.Network(f).order(args.order, seed=i) for i, f in enumerate(formulas[:4])]
    out = {
        "metric": "exact counts/sec + contraction HBM GB/s; learned vs greedy order wall-time",
        "value": round(value, 4), "unit": "counts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "u32" if args.wide_rns else "i8",
        "data": "synthetic",
        "config": {"workload": workload, "batch": args.batch, "n": args.n if args.workload == "cvc" else None,
                   "order": args.order, "moduli": k_primes, "residue_mode": mode},
        "roofline": roofline,
        "hbm_roofline_stream": roofline_of("stream", prof["stream"]) if prof["stream"]["launches"] else None,
        "kernel_classes": per_class,
        "learned_vs_greedy": lvg,
        "plan_max_rank": [p.stats["max_rank"] for p in plans],
        "plan_chosen": [p.stats["chosen"] for p in plans],
    }
    if not args.no_cpu_baseline:
        p0 = plans[0]
        out["cpu_baseline"] = cpu_baseline(formulas[0], p0.steps(), args.cpu_seconds)
        log("cpu baseline done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
