"""Pins for the binary64 tuner-network oracle: autograd, finite differences, the Adam
reference implementation in torch, and closed-form special cases."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp

D_IN, H, C = 24, 64, 9


def params(seed, scale=0.3):
    shapes = dict(W1=(D_IN, H), b1=(H,), W2=(H, H), b2=(H,), W3=(H, C), b3=(C,))
    out = {}
    for s, (k, sh) in enumerate(shapes.items()):
        out[k] = scale * synth.uniform_pm1(seed, 100 + s, int(np.prod(sh))).reshape(sh)
    return out


def data(seed, B=17):
    X = synth.uniform_pm1(seed, 1, B * D_IN).reshape(B, D_IN)
    T = synth.uniform_pm1(seed, 2, B * C).reshape(B, C)
    M = (synth.uniform01(seed, 3, B * C) < 0.8).astype(np.float64).reshape(B, C)
    M[0, 0] = 1.0
    return X, T, M


@pytest.mark.parametrize("seed", range(3))
def test_backward_matches_torch_autograd(seed):
    p = params(seed)
    X, T, M = data(seed)
    acts = mlp.forward(p, X)
    g = mlp.backward(p, acts, T, M)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    Xt, Tt, Mt = (torch.tensor(a, dtype=torch.float64) for a in (X, T, M))
    h1 = torch.relu(Xt @ tp["W1"] + tp["b1"])
    h2 = torch.relu(h1 @ tp["W2"] + tp["b2"])
    P = h2 @ tp["W3"] + tp["b3"]
    L = (Mt * (P - Tt) ** 2).sum() / Mt.sum()
    L.backward()
    assert abs(L.item() - mlp.loss(acts["P"], T, M)) < 1e-14
    for k in p:
        ref = tp[k].grad.numpy()
        assert np.allclose(g[k], ref, rtol=1e-12, atol=1e-14), k


def test_backward_matches_central_differences():
    p = params(7)
    X, T, M = data(7, B=5)
    g = mlp.backward(p, mlp.forward(p, X), T, M)
    eps = 1e-6
    for k in p:
        flat = p[k].ravel()
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k].ravel()[idx] += eps
            lp = mlp.loss(mlp.forward(q, X)["P"], T, M)
            q[k].ravel()[idx] -= 2 * eps
            lm = mlp.loss(mlp.forward(q, X)["P"], T, M)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[k].ravel()[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_forward_special_cases():
    p = params(3)
    X, _, _ = data(3)
    z = {k: np.zeros_like(v) for k, v in p.items()}
    z["b3"] = p["b3"]
    assert np.array_equal(mlp.forward(z, X)["P"], np.broadcast_to(p["b3"], (X.shape[0], C)))
    # with zero biases a ReLU network is positively homogeneous: f(cX) = c f(X)
    nb = dict(p, b1=np.zeros(H), b2=np.zeros(H), b3=np.zeros(C))
    assert np.allclose(mlp.forward(nb, 4.0 * X)["P"], 4.0 * mlp.forward(nb, X)["P"], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("steps", [1, 3])
def test_adam_matches_torch_optim(steps):
    p = params(11)
    X, T, M = data(11)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(vv) for k, vv in p.items()}
    tp = [torch.tensor(p[k], dtype=torch.float64, requires_grad=True) for k in p]
    opt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    cur = p
    for s in range(1, steps + 1):
        g = mlp.backward(cur, mlp.forward(cur, X), T, M)
        cur, m, v = mlp.adam_step(cur, g, m, v, s, lr=1e-2)
        opt.zero_grad()
        for t, k in zip(tp, p):
            t.grad = torch.tensor(g[k], dtype=torch.float64)
        opt.step()
    for t, k in zip(tp, p):
        assert np.allclose(cur[k], t.detach().numpy(), rtol=1e-12, atol=1e-15), k
