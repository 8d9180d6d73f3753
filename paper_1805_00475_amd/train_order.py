"""Train the order-scoring perceptron on the GPU with the library's kernels.

    python -m paper_1805_00475_amd.train_order [--train 256] [--epochs 10]
        [--out paper_1805_00475_amd/models/order_mlp.npy]

Training data are imitation traces: monotone 1-in-3 instances with n drawn
uniformly in [100, 250] and m = round(0.66 n) (Sec. 3.2 workload family),
each ordered by the library's judge (the cheapest of greedy, randomized
bisection and Girvan-Newman plans under the cost model); along the judged
order, every state contributes its candidate pairs with the pairs the
teacher contracts next marked. The listwise loss, its gradients and Adam run
in the library's HIP kernels; this script only moves arrays.

    python -m paper_1805_00475_amd.train_order --evaluate MODEL [--heldout 256]

compares learned, greedy and judged orders on held-out instances by the
predicted cost of their plans and by host ordering time.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_MODEL = os.path.join(HERE, "models", "order_mlp.npy")


def _trace_one(args):
    i, split, stride = args
    import instances as I
    from paper_1805_00475_amd import tn
    f = I.learned_instance(i, split)
    net = tn.Network(f)
    teacher = net.order("best", seed=i)
    X, lab, g = tn.trace(net, teacher)
    keep = list(range(0, len(g) - 1, stride))
    xs, ls, sizes = [], [], []
    for k in keep:
        a, b = g[k], g[k + 1]
        xs.append(X[a:b])
        ls.append(lab[a:b])
        sizes.append(b - a)
    return np.concatenate(xs), np.concatenate(ls), np.array(sizes, dtype=np.int64), teacher.stats["chosen"]


def build_dataset(count, split="train", stride=2, workers=16):
    """Concatenated (features, labels, group offsets) of ``count`` instances."""
    ctx = __import__("multiprocessing").get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        parts = list(ex.map(_trace_one, [(i, split, stride) for i in range(count)]))
    X = np.concatenate([p[0] for p in parts]).astype(np.float32)
    L = np.concatenate([p[1] for p in parts]).astype(np.uint8)
    sizes = np.concatenate([p[2] for p in parts])
    G = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    teachers = {}
    for p in parts:
        teachers[p[3]] = teachers.get(p[3], 0) + 1
    return X, L, G, teachers


def init_params(seed=0):
    """He-style initial parameters in the library's packing: W1 [128 x 10],
    b1, W2 [128 x 128], b2, w3 [128], b3."""
    r = np.random.default_rng(seed)
    F, H = 10, 128
    parts = [r.normal(0, math.sqrt(2.0 / F), H * F), np.zeros(H), r.normal(0, math.sqrt(2.0 / H), H * H),
             np.zeros(H), r.normal(0, math.sqrt(1.0 / H), H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def train(X, L, G, epochs=10, lr=2e-3, batch_groups=64, seed=0, log=print):
    """Adam on the GPU kernels; returns the trained parameters (numpy)."""
    import torch
    from paper_1805_00475_amd import tn
    rng = np.random.default_rng(seed)
    p0 = init_params(seed)
    dev = "cuda"
    P = torch.from_numpy(p0).to(dev)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    Xd = torch.from_numpy(X).to(dev)
    Ld = torch.from_numpy(L).to(dev)
    n_groups = len(G) - 1
    chunks = [(a, min(a + batch_groups, n_groups)) for a in range(0, n_groups, batch_groups)]
    max_rows = max(int(G[b] - G[a]) for a, b in chunks)
    f = dict(dtype=torch.float32, device=dev)
    h1, h2 = torch.empty(max_rows, 128, **f), torch.empty(max_rows, 128, **f)
    y, dy = torch.empty(max_rows, **f), torch.empty(max_rows, **f)
    dz2, dz1 = torch.empty(max_rows, 128, **f), torch.empty(max_rows, 128, **f)
    grad, loss = torch.empty_like(P), torch.empty(1, **f)
    step = 0
    history = []
    for ep in range(epochs):
        order = rng.permutation(len(chunks))
        tot = 0.0
        for ci in order:
            a, b = chunks[ci]
            r0, r1 = int(G[a]), int(G[b])
            gr = torch.from_numpy((G[a:b + 1] - G[a]).astype(np.int32)).to(dev)
            x = Xd[r0:r1]
            tn.mlp_forward(P, x, h1, h2, y)
            tn.mlp_backward(P, x, h1, h2, y, Ld[r0:r1], gr, grad, dz2, dz1, dy, loss)
            step += 1
            tn.mlp_adam(P, grad, m, v, step, lr=lr)
            tot += loss.item() * (b - a)
        history.append(tot / n_groups)
        log(f"[train] epoch {ep + 1}/{epochs} mean loss {history[-1]:.4f}")
    return P.cpu().numpy(), history


def _eval_one(args):
    i, split, model_path = args
    import instances as I
    from paper_1805_00475_amd import tn
    model = tn.Model.load_file(model_path)
    f = I.learned_instance(i, split)
    net = tn.Network(f)
    out = {"index": i, "n": f.n_vars}
    for kind in ("greedy", "learned_raw", "best", "learned"):
        t = time.perf_counter()
        try:
            p = net.order(kind, seed=i, model=model if "learned" in kind else None)
            out[kind] = {"log2_cost": p.stats["log2_cost"], "max_rank": p.stats["max_rank"],
                         "chosen": p.stats["chosen"], "fallback": p.stats["fallback"]}
        except tn.TNError as e:
            out[kind] = {"error": str(e)}
        out[kind]["order_ms"] = 1000 * (time.perf_counter() - t)
    return out


def evaluate(model_path, count=256, split="heldout", workers=16):
    ctx = __import__("multiprocessing").get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        rows = list(ex.map(_eval_one, [(i, split, model_path) for i in range(count)]))

    def cost(r, k):
        return r[k].get("log2_cost", math.inf)
    lg = [cost(r, "learned_raw") for r in rows]
    gr = [cost(r, "greedy") for r in rows]
    be = [cost(r, "best") for r in rows]
    summary = {
        "instances": count,
        "learned_beats_greedy": sum(a < b for a, b in zip(lg, gr)) / count,
        "learned_within_best": sum(a <= b + 1e-9 for a, b in zip(lg, be)) / count,
        "greedy_over_rank_cap": sum(math.isinf(x) for x in gr) / count,
        "median_log2_cost": {"greedy": float(np.median(gr)), "learned_raw": float(np.median(lg)),
                             "best": float(np.median(be))},
        "mean_order_ms": {k: float(np.mean([r[k]["order_ms"] for r in rows]))
                          for k in ("greedy", "learned_raw", "best", "learned")},
        "judged_learned_fallback_rate": float(np.mean([bool(r["learned"].get("fallback", True)) for r in rows])),
    }
    return summary, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=256)
    ap.add_argument("--stride", type=int, default=2)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--evaluate", default=None)
    ap.add_argument("--heldout", type=int, default=256)
    args = ap.parse_args()
    if args.evaluate:
        s, _ = evaluate(args.evaluate, args.heldout)
        print(json.dumps(s))
        return
    t = time.time()
    X, L, G, teachers = build_dataset(args.train, "train", args.stride)
    print(f"[train] dataset: {len(L)} rows, {len(G) - 1} states, teachers {teachers}, "
          f"{time.time() - t:.1f}s", flush=True)
    params, hist = train(X, L, G, args.epochs, args.lr, log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, params.astype(np.float32))
    meta = {"train_instances": args.train, "state_stride": args.stride, "epochs": args.epochs, "lr": args.lr,
            "rows": int(len(L)), "states": int(len(G) - 1), "teachers": teachers, "loss_history": hist}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    print("[train] saved", args.out, flush=True)
    s, _ = evaluate(args.out, args.heldout)
    print(json.dumps(s), flush=True)


if __name__ == "__main__":
    main()
