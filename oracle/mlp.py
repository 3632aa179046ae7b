"""FP64 reference of the residual-corrector network (oracle, test infrastructure).

Not part of the paper: a small multilayer perceptron g(xi) = W3 s(W2 s(W1 xi + b1) + b2) + b3
with s(z) = z / (1 + exp(-z)) (SiLU), layer sizes 3 -> 64 -> 64 -> 1, trained by Adam
(Kingma and Ba 2015) on the mean squared error against the functional Tucker residual.
This module is plain float64 NumPy: forward pass, back-propagation written out layer by
layer, and the Adam update with bias correction.
"""
from __future__ import annotations

import numpy as np

LAYERS = (3, 64, 64, 1)


def init_params(seed: int, layers=LAYERS):
    """Xavier-uniform weights (bound sqrt(6 / (fan_in + fan_out))), zero biases."""
    rng = np.random.default_rng(seed)
    params = {}
    for l in range(len(layers) - 1):
        fi, fo = layers[l], layers[l + 1]
        b = np.sqrt(6.0 / (fi + fo))
        params[f"W{l+1}"] = rng.uniform(-b, b, size=(fo, fi))
        params[f"b{l+1}"] = np.zeros(fo)
    return params


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params, x):
    """Returns (y (B,), cache)."""
    x = np.asarray(x, np.float64)
    z1 = x @ params["W1"].T + params["b1"]
    a1 = silu(z1)
    z2 = a1 @ params["W2"].T + params["b2"]
    a2 = silu(z2)
    y = (a2 @ params["W3"].T + params["b3"])[:, 0]
    return y, (x, z1, a1, z2, a2)


def loss_and_grads(params, x, t):
    """MSE loss mean((y - t)^2) and its gradients with respect to every parameter."""
    y, (x, z1, a1, z2, a2) = forward(params, x)
    B = x.shape[0]
    d = y - np.asarray(t, np.float64)
    loss = float(np.mean(d * d))
    dy = (2.0 / B) * d[:, None]                 # (B, 1)
    g = {"W3": dy.T @ a2, "b3": dy.sum(axis=0)}
    dz2 = (dy @ params["W3"]) * silu_grad(z2)   # (B, 64)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ params["W2"]) * silu_grad(z1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return loss, g


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        for k in params:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * grads[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * grads[k] ** 2
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            params[k] = params[k] - self.lr * mh / (np.sqrt(vh) + self.eps)
        return params


def n_params(layers=LAYERS) -> int:
    return sum(layers[l] * layers[l + 1] + layers[l + 1] for l in range(len(layers) - 1))


PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(params) -> np.ndarray:
    """Parameters in the library's flat order: W1 (64x3), b1, W2 (64x64), b2, W3 (1x64), b3."""
    return np.concatenate([np.asarray(params[k], np.float64).reshape(-1) for k in PARAM_ORDER])


def unflatten(flat) -> dict:
    flat = np.asarray(flat, np.float64)
    shapes = {"W1": (64, 3), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (1, 64), "b3": (1,)}
    out, o = {}, 0
    for k in PARAM_ORDER:
        size = int(np.prod(shapes[k]))
        out[k] = flat[o:o + size].reshape(shapes[k]).copy()
        o += size
    return out


def train(params, xi, target, steps, batch, seed, lr=1e-3):
    """Adam on mean squared error with minibatches drawn by sampler.batch_indices."""
    from .sampler import batch_indices
    params = {k: v.copy() for k, v in params.items()}
    opt = Adam(params, lr=lr)
    losses = []
    for s in range(steps):
        idx = batch_indices(seed, s, batch, xi.shape[0])
        loss, g = loss_and_grads(params, xi[idx], target[idx])
        params = opt.step(params, g)
        losses.append(loss)
    return params, losses
