"""Pins of the float64 perceptron reference: central finite differences of
the loss against the analytic gradient, a closed form of the loss, Adam
against its textbook recurrence, and a planted mistake that the
finite-difference check must catch."""
import numpy as np
import pytest

from oracle import mlp


def _problem(seed, n=40, groups=6):
    r = np.random.default_rng(seed)
    X = r.normal(0, 1, (n, mlp.F))
    cuts = np.sort(r.choice(np.arange(1, n), size=groups - 1, replace=False))
    g = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    lab = np.zeros(n, dtype=np.uint8)
    for k in range(groups):
        a, b = g[k], g[k + 1]
        lab[r.integers(a, b)] = 1
        if b - a > 2 and r.random() < 0.5:
            lab[r.integers(a, b)] = 1
    return X, lab, g


def _fd(p, X, lab, g, idx, eps=1e-6):
    out = []
    for i in idx:
        q = p.copy()
        q[i] += eps
        lp = mlp.loss(q, X, lab, g)
        q[i] -= 2 * eps
        lm = mlp.loss(q, X, lab, g)
        out.append((lp - lm) / (2 * eps))
    return np.array(out)


def _sample_indices(seed, k=60):
    r = np.random.default_rng(seed)
    offs = [0, mlp.H * mlp.F, mlp.H * mlp.F + mlp.H, mlp.H * mlp.F + mlp.H + mlp.H * mlp.H,
            mlp.H * mlp.F + 2 * mlp.H + mlp.H * mlp.H, mlp.N_PARAMS - 1 - mlp.H, mlp.N_PARAMS - 1]
    idx = set(r.integers(0, mlp.N_PARAMS, k).tolist()) | {mlp.N_PARAMS - 1}
    for a, b in zip(offs, offs[1:] + [mlp.N_PARAMS]):
        idx |= set(r.integers(a, max(a + 1, b), 4).tolist())
    return sorted(i for i in idx if i < mlp.N_PARAMS)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_finite_differences(seed):
    X, lab, g = _problem(seed)
    p = mlp.init_params(seed)
    idx = _sample_indices(seed)
    an = mlp.grad(p, X, lab, g)[idx]
    fd = _fd(p, X, lab, g, idx)
    assert np.allclose(an, fd, rtol=1e-5, atol=1e-8)


def test_loss_closed_form_with_constant_scores():
    # W2 = 0 and w3 = 0 make every score b3: L_g = log n_g - log n_pos(g)
    X, lab, g = _problem(5)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(mlp.init_params(5))
    p = mlp.pack(W1, b1, 0 * W2, b2, 0 * w3, 0.7)
    want = np.mean([np.log(g[k + 1] - g[k]) - np.log(lab[g[k]:g[k + 1]].sum()) for k in range(len(g) - 1)])
    assert mlp.loss(p, X, lab, g) == pytest.approx(want, rel=1e-12)


def test_adam_against_recurrence():
    r = np.random.default_rng(3)
    p = r.normal(size=7)
    m = np.zeros(7)
    v = np.zeros(7)
    pp = p.copy()
    for t in range(1, 4):
        g = r.normal(size=7)
        p, m, v = mlp.adam(p, g, m, v, t, lr=0.01)
        # the first step of Adam moves every coordinate by lr * sign(g)
        if t == 1:
            assert np.allclose(pp - p, 0.01 * np.sign(g), rtol=1e-6)


def test_planted_missing_relu_mask_is_caught(monkeypatch):
    X, lab, g = _problem(7)
    p = mlp.init_params(7)
    orig = mlp.grad

    def bad(p, X, lab, g):
        W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
        y, h1, h2 = mlp.forward(p, X)
        G = len(g) - 1
        dy = np.zeros_like(y)
        for k in range(G):
            a, b = g[k], g[k + 1]
            pos = lab[a:b] > 0
            e = np.exp(y[a:b] - y[a:b].max())
            dy[a:b] = (e / e.sum() - np.where(pos, e, 0) / e[pos].sum()) / G
        dz2 = np.outer(dy, w3) * (h2 > 0)
        dz1 = dz2 @ W2  # relu mask of layer 1 dropped
        return mlp.pack(dz1.T @ X, dz1.sum(0), dz2.T @ h1, dz2.sum(0), h2.T @ dy, dy.sum())

    idx = _sample_indices(7)
    assert np.allclose(orig(p, X, lab, g)[idx], _fd(p, X, lab, g, idx), rtol=1e-5, atol=1e-8)
    assert not np.allclose(bad(p, X, lab, g)[idx], _fd(p, X, lab, g, idx), rtol=1e-5, atol=1e-8)
