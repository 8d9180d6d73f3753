"""float64 reference of the order-scoring perceptron and its gradients.

Test infrastructure only. Parameter packing (the library's interface, restated
here): W1 [128 x 10], b1 [128], W2 [128 x 128], b2 [128], w3 [128], b3.

    h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3

Listwise loss over groups of rows (the candidate pairs of one state): with
P the rows labelled 1,
    L_g = log sum_{i in g} exp(y_i) - log sum_{i in g, i in P} exp(y_i),
and L = mean over groups. Its derivative in y_i is
    (softmax over the group)_i - (softmax over the group's positives)_i
(the second term is 0 for unlabelled rows), divided by the number of groups.
Backpropagation then follows the chain rule through the three layers.

Also: the candidate-pair features used by the learned order, recomputed
from label sets along a merge sequence.
"""
from __future__ import annotations

import numpy as np

F = 10
H = 128
N_PARAMS = H * F + H + H * H + H + H + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def forward(p, X):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, h1, h2


def loss(p, X, labels, groups):
    y, _, _ = forward(p, X)
    G = len(groups) - 1
    total = 0.0
    for g in range(G):
        a, b = groups[g], groups[g + 1]
        yy = y[a:b]
        pos = np.asarray(labels[a:b]) > 0
        if b <= a or not pos.any():
            continue
        m = yy.max()
        total += (m + np.log(np.exp(yy - m).sum())) - (m + np.log(np.exp(yy[pos] - m).sum()))
    return total / G


def grad(p, X, labels, groups):
    """Analytic gradient of ``loss`` with respect to the packed parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    y, h1, h2 = forward(p, X)
    G = len(groups) - 1
    dy = np.zeros_like(y)
    for g in range(G):
        a, b = groups[g], groups[g + 1]
        pos = np.asarray(labels[a:b]) > 0
        if b <= a or not pos.any():
            continue
        yy = y[a:b]
        e = np.exp(yy - yy.max())
        sa = e / e.sum()
        sp = np.where(pos, e, 0.0)
        sp = sp / sp.sum()
        dy[a:b] = (sa - sp) / G
    dw3 = h2.T @ dy
    db3 = dy.sum()
    dz2 = np.outer(dy, w3) * (h2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (h1 > 0)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) with bias correction; returns new p, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-style random initial parameters."""
    r = np.random.default_rng(seed)
    W1 = r.normal(0, np.sqrt(2.0 / F), (H, F))
    W2 = r.normal(0, np.sqrt(2.0 / H), (H, H))
    w3 = r.normal(0, np.sqrt(1.0 / H), H)
    return pack(W1, np.zeros(H), W2, np.zeros(H), w3, 0.0)


# ---------------------------------------------------------------- features
def pair_features(live, u, v):
    """Features of merging live tensors u and v; ``live`` maps id -> label set.

    With rA >= rB (ties: the larger neighbour count first), s shared labels,
    rC = rA + rB - 2s, dA, dB the numbers of other live tensors sharing a
    label with each, c the number of tensors sharing a label with both:
    rA/32, rB/32, s/32, rC/32, (rC - rA)/8, dA/16, dB/16, c/8,
    (rA + rB - s)/48, [s == rB].
    """
    def nbrs(x):
        return {y for y in live if y != x and live[y] & live[x]}
    nu, nv = nbrs(u), nbrs(v)
    ru, rv, du, dv = len(live[u]), len(live[v]), len(nu), len(nv)
    if rv > ru or (rv == ru and dv > du):
        u, v, ru, rv, du, dv, nu, nv = v, u, rv, ru, dv, du, nv, nu
    s = len(live[u] & live[v])
    rc = ru + rv - 2 * s
    common = len((nu - {v}) & (nv - {u}))
    return np.array([ru / 32, rv / 32, s / 32, rc / 32, (rc - ru) / 8, du / 16, dv / 16, common / 8,
                     (ru + rv - s) / 48, 1.0 if s == rv else 0.0], dtype=np.float64)


def trace(label_sets, merges):
    """Rows (features, label) of every state along ``merges``; labels mark
    pairs that ``merges`` contracts while both are alive. Returns a list of
    groups, each a list of ((lo, hi), features, label)."""
    live = {i: frozenset(s) for i, s in enumerate(label_sets)}
    nid = len(label_sets)
    partner = {}
    for a, b in merges:
        partner[a] = b
        partner[b] = a
    groups = []
    for a, b in merges:
        rows = []
        ids = sorted(live)
        seen = False
        for i, u in enumerate(ids):
            for v in ids[i + 1:]:
                if live[u] & live[v]:
                    rows.append(((u, v), pair_features(live, u, v), 1 if partner.get(u) == v else 0))
                    if (u, v) == (min(a, b), max(a, b)):
                        seen = True
        if not seen:
            rows.append(((min(a, b), max(a, b)), pair_features(live, a, b), 1))
        groups.append(rows)
        live[nid] = live.pop(a) ^ live.pop(b)
        nid += 1
    return groups
