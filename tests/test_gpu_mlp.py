"""The tuner network's HIP kernels against the binary64 oracle: forward, gradients, Adam,
inference argmin; determinism and a decreasing loss."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp as ref
from paper_1112_5588_amd import _lib as L

pytestmark = pytest.mark.gpu

D_IN, H = 24, 64


def init(d_out, seed, scale=0.3):
    shapes = dict(W1=(D_IN, H), b1=(H,), W2=(H, H), b2=(H,), W3=(H, d_out), b3=(d_out,))
    p = {k: scale * synth.uniform_pm1(seed, 100 + s, int(np.prod(sh))).reshape(sh) for s, (k, sh) in enumerate(shapes.items())}
    flat = np.concatenate([p[k].ravel() for k in shapes]).astype(np.float32)
    # the oracle sees exactly the float32 values the GPU uses
    p32 = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    assert flat.size == L.mlp_param_count(D_IN, d_out)
    return p32, torch.from_numpy(flat).cuda()


def data(B, d_out, seed):
    X = synth.uniform_pm1(seed, 1, B * D_IN).reshape(B, D_IN).astype(np.float32)
    T = synth.uniform_pm1(seed, 2, B * d_out).reshape(B, d_out).astype(np.float32)
    M = (synth.uniform01(seed, 3, B * d_out) < 0.85).astype(np.float32).reshape(B, d_out)
    M[0, 0] = 1
    return X, T, M


def unflat(g, d_out):
    sizes = [("W1", D_IN * H, (D_IN, H)), ("b1", H, (H,)), ("W2", H * H, (H, H)), ("b2", H, (H,)),
             ("W3", H * d_out, (H, d_out)), ("b3", d_out, (d_out,))]
    out, o = {}, 0
    for k, n, sh in sizes:
        out[k] = g[o:o + n].reshape(sh)
        o += n
    return out


def rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("B,d_out", [(1, 22), (64, 22), (200, 22), (777, 9), (130, 64)])
def test_forward_and_gradients_match_oracle(B, d_out):
    p, dp = init(d_out, seed=B)
    X, T, M = data(B, d_out, seed=B + 1)
    dX, dT, dM = (torch.from_numpy(a).cuda() for a in (X, T, M))
    P = torch.empty((B, d_out), dtype=torch.float32, device="cuda")
    L.mlp_forward(dp, D_IN, d_out, dX, P)
    acts = ref.forward(p, X.astype(np.float64))
    assert rel(P.cpu().numpy(), acts["P"]) < 1e-5
    n = dp.numel()
    grad = torch.empty(n, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    work = torch.empty(L.mlp_workspace_size(D_IN, d_out, B) // 4 + 1, dtype=torch.float32, device="cuda")
    L.mlp_backward(dp, D_IN, d_out, dX, dT, dM, grad, loss, work)
    g_ref = ref.backward(p, acts, T.astype(np.float64), M.astype(np.float64))
    g = unflat(grad.cpu().numpy(), d_out)
    for k in g_ref:
        assert rel(g[k], g_ref[k]) < 1e-4, k
    assert abs(loss.item() - ref.loss(acts["P"], T, M)) <= 1e-5 * max(1.0, ref.loss(acts["P"], T, M))
    # deterministic: a second evaluation is bitwise identical
    grad2 = torch.empty_like(grad)
    L.mlp_backward(dp, D_IN, d_out, dX, dT, dM, grad2, None, work)
    assert torch.equal(grad, grad2)


def test_adam_matches_oracle():
    d_out = 22
    p, dp = init(d_out, seed=5)
    X, T, M = data(300, d_out, seed=6)
    dX, dT, dM = (torch.from_numpy(a).cuda() for a in (X, T, M))
    n = dp.numel()
    grad = torch.empty(n, dtype=torch.float32, device="cuda")
    work = torch.empty(L.mlp_workspace_size(D_IN, d_out, 300) // 4 + 1, dtype=torch.float32, device="cuda")
    m = torch.zeros(n, dtype=torch.float32, device="cuda")
    v = torch.zeros(n, dtype=torch.float32, device="cuda")
    pm = {k: np.zeros_like(a) for k, a in p.items()}
    pv = {k: np.zeros_like(a) for k, a in p.items()}
    cur = p
    for step in range(1, 4):
        L.mlp_backward(dp, D_IN, d_out, dX, dT, dM, grad, None, work)
        # oracle step on the GPU's own gradient, so only the update rule is compared
        g = {k: a.astype(np.float64) for k, a in unflat(grad.cpu().numpy(), d_out).items()}
        L.mlp_adam_step(dp, grad, m, v, step, lr=1e-2)
        cur, pm, pv = ref.adam_step(cur, g, pm, pv, step, lr=1e-2)
        got = unflat(dp.cpu().numpy(), d_out)
        for k in cur:
            assert np.allclose(got[k], cur[k], rtol=1e-5, atol=1e-6), (step, k)
        cur = {k: got[k].astype(np.float64) for k in cur}


def test_infer_argmin_and_margin():
    d_out = 22
    p, dp = init(d_out, seed=8)
    X, _, _ = data(500, d_out, seed=9)
    scale = (0.5 + synth.uniform01(10, 1, d_out)).astype(np.float32)
    shift = synth.uniform_pm1(10, 2, d_out).astype(np.float32)
    valid = np.ones(d_out, np.float32)
    valid[[3, 7]] = 0
    idx = torch.empty(500, dtype=torch.int32, device="cuda")
    mg = torch.empty(500, dtype=torch.float32, device="cuda")
    L.mlp_infer(dp, D_IN, d_out, torch.from_numpy(X).cuda(), torch.from_numpy(scale).cuda(),
                torch.from_numpy(shift).cuda(), torch.from_numpy(valid).cuda(), idx, mg)
    P = ref.forward(p, X.astype(np.float64))["P"] * scale + shift
    P[:, valid == 0] = np.inf
    srt = np.sort(P, axis=1)
    got = idx.cpu().numpy()
    # where the two best predictions are not within float32 noise, the argmin is unique
    clear = srt[:, 1] - srt[:, 0] > 1e-4
    assert np.array_equal(got[clear], P.argmin(axis=1)[clear])
    assert np.all(valid[got] == 1)
    assert np.allclose(mg.cpu().numpy()[clear], (srt[:, 1] - srt[:, 0])[clear], atol=1e-4)


def test_training_reduces_loss():
    d_out = 9
    _, dp = init(d_out, seed=12, scale=0.1)
    X, _, _ = data(1024, d_out, seed=13)
    # a learnable target: a fixed random linear map of the features
    Wt = synth.uniform_pm1(14, 1, D_IN * d_out).reshape(D_IN, d_out)
    T = (X @ Wt).astype(np.float32) / 3
    M = np.ones_like(T)
    dX, dT, dM = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (X, T, M))
    n = dp.numel()
    grad = torch.empty(n, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    work = torch.empty(L.mlp_workspace_size(D_IN, d_out, 1024) // 4 + 1, dtype=torch.float32, device="cuda")
    m, v = torch.zeros_like(grad), torch.zeros_like(grad)
    losses = []
    for step in range(1, 301):
        L.mlp_backward(dp, D_IN, d_out, dX, dT, dM, grad, loss, work)
        L.mlp_adam_step(dp, grad, m, v, step, lr=3e-3)
        if step in (1, 300):
            losses.append(loss.item())
    assert losses[1] < 0.1 * losses[0], losses
