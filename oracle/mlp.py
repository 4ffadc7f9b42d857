"""Binary64 oracle of the tuner network -- TEST INFRASTRUCTURE ONLY.

The learned tuner maps matrix features to a predicted (standardised) run time per kernel
configuration with a three-layer perceptron:

    Z1 = X W1 + b1,  H1 = relu(Z1)
    Z2 = H1 W2 + b2, H2 = relu(Z2)
    P  = H2 W3 + b3

Weights are stored (fan_in, fan_out) row-major.  The loss is the masked mean squared error
L = sum(M * (P - T)^2) / sum(M), the mask M marking the (matrix, configuration) pairs that
have a label.  Training uses Adam (Kingma and Ba, "Adam: a method for stochastic
optimization", ICLR 2015) with bias correction.  relu'(0) is taken as 0.

Everything here is written from those definitions in numpy binary64; matrix products are
the library primitive.
"""
from __future__ import annotations

import numpy as np


def forward(params: dict, X: np.ndarray) -> dict:
    """Returns the activations of every layer (binary64)."""
    X = np.asarray(X, np.float64)
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3"))
    Z1 = X @ W1 + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2 + b2
    H2 = np.maximum(Z2, 0.0)
    P = H2 @ W3 + b3
    return dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2, P=P)


def loss(P: np.ndarray, T: np.ndarray, M: np.ndarray) -> float:
    """Masked mean squared error."""
    M = np.asarray(M, np.float64)
    d = np.asarray(P, np.float64) - np.asarray(T, np.float64)
    return float((M * d * d).sum() / M.sum())


def backward(params: dict, acts: dict, T: np.ndarray, M: np.ndarray) -> dict:
    """Gradients of the masked MSE with respect to every parameter (chain rule)."""
    M = np.asarray(M, np.float64)
    dP = 2.0 * M * (acts["P"] - np.asarray(T, np.float64)) / M.sum()
    W2, W3 = np.asarray(params["W2"], np.float64), np.asarray(params["W3"], np.float64)
    g = {}
    g["W3"] = acts["H2"].T @ dP
    g["b3"] = dP.sum(axis=0)
    dZ2 = (dP @ W3.T) * (acts["Z2"] > 0)
    g["W2"] = acts["H1"].T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * (acts["Z1"] > 0)
    g["W1"] = acts["X"].T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_step(params: dict, grads: dict, m: dict, v: dict, step: int, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> tuple[dict, dict, dict]:
    """One Adam update at (1-based) ``step``; returns new params, first and second moments."""
    newp, newm, newv = {}, {}, {}
    for k in params:
        g = np.asarray(grads[k], np.float64)
        mk = beta1 * np.asarray(m[k], np.float64) + (1.0 - beta1) * g
        vk = beta2 * np.asarray(v[k], np.float64) + (1.0 - beta2) * g * g
        mhat = mk / (1.0 - beta1 ** step)
        vhat = vk / (1.0 - beta2 ** step)
        newp[k] = np.asarray(params[k], np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
        newm[k], newv[k] = mk, vk
    return newp, newm, newv
