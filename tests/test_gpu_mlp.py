"""The perceptron's HIP kernels (forward, listwise-loss backward, Adam)
against the float64 oracle; a few GPU training steps lower the loss."""
import numpy as np
import pytest

from oracle import mlp
from paper_1805_00475_amd import tn

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _problem(seed, n, groups):
    r = np.random.default_rng(seed)
    X = r.normal(0, 1, (n, mlp.F)).astype(np.float32)
    cuts = np.sort(r.choice(np.arange(1, n), size=groups - 1, replace=False))
    g = np.concatenate([[0], cuts, [n]]).astype(np.int32)
    lab = np.zeros(n, dtype=np.uint8)
    for k in range(groups):
        lab[r.integers(g[k], g[k + 1], size=1 + (k % 3))] = 1
    return X, lab, g


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _buffers(n):
    import torch
    f = dict(dtype=torch.float32, device="cuda")
    return (torch.empty(n, mlp.H, **f), torch.empty(n, mlp.H, **f), torch.empty(n, **f),
            torch.empty(mlp.N_PARAMS, **f), torch.empty(n, mlp.H, **f), torch.empty(n, mlp.H, **f),
            torch.empty(n, **f), torch.empty(1, **f))


@pytest.mark.parametrize("n,groups", [(1, 1), (300, 7), (5000, 120)])
def test_forward_backward_vs_oracle(n, groups):
    import torch
    _say(f"mlp fwd/bwd n={n} groups={groups}")
    X, lab, g = _problem(n, n, groups)
    p = mlp.init_params(n).astype(np.float32)
    h1, h2, y, grad, dz2, dz1, dy, loss = _buffers(n)
    P, Xd, Ld, Gd = _dev(p), _dev(X), _dev(lab), _dev(g)
    tn.mlp_forward(P, Xd, h1, h2, y)
    tn.mlp_backward(P, Xd, h1, h2, y, Ld, Gd, grad, dz2, dz1, dy, loss)
    torch.cuda.synchronize()
    p64 = p.astype(np.float64)
    want_y, _, _ = mlp.forward(p64, X.astype(np.float64))
    got_y = y.cpu().numpy()
    assert np.allclose(got_y, want_y, rtol=1e-4, atol=1e-4 * max(1.0, np.abs(want_y).max()))
    assert loss.item() == pytest.approx(mlp.loss(p64, X.astype(np.float64), lab, g), rel=1e-4, abs=1e-5)
    want_g = mlp.grad(p64, X.astype(np.float64), lab, g)
    got_g = grad.cpu().numpy()
    scale = np.abs(want_g).max()
    assert np.allclose(got_g, want_g, rtol=2e-3, atol=2e-4 * scale)


def test_adam_vs_oracle():
    import torch
    _say("adam")
    r = np.random.default_rng(1)
    p = r.normal(size=mlp.N_PARAMS).astype(np.float32)
    P = _dev(p)
    m = torch.zeros(mlp.N_PARAMS, device="cuda")
    v = torch.zeros(mlp.N_PARAMS, device="cuda")
    pp, mm, vv = p.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for t in range(1, 4):
        g = r.normal(size=mlp.N_PARAMS).astype(np.float32)
        tn.mlp_adam(P, _dev(g), m, v, t, lr=1e-2)
        pp, mm, vv = mlp.adam(pp, g.astype(np.float64), mm, vv, t, lr=1e-2)
    torch.cuda.synchronize()
    assert np.allclose(P.cpu().numpy(), pp, rtol=1e-5, atol=1e-5)


def test_training_steps_lower_the_loss():
    import torch
    _say("training steps")
    X, lab, g = _problem(9, 4000, 100)
    # make the positives learnable: their first feature is shifted up
    X[lab > 0, 0] += 2.0
    p = mlp.init_params(9).astype(np.float32)
    h1, h2, y, grad, dz2, dz1, dy, loss = _buffers(len(X))
    P, Xd, Ld, Gd = _dev(p), _dev(X), _dev(lab), _dev(g)
    m = torch.zeros(mlp.N_PARAMS, device="cuda")
    v = torch.zeros(mlp.N_PARAMS, device="cuda")
    losses = []
    for t in range(1, 61):
        tn.mlp_forward(P, Xd, h1, h2, y)
        tn.mlp_backward(P, Xd, h1, h2, y, Ld, Gd, grad, dz2, dz1, dy, loss)
        losses.append(loss.item())
        tn.mlp_adam(P, grad, m, v, t, lr=3e-3)
    assert losses[-1] < 0.5 * losses[0]
