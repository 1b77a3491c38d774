"""Residual-network training reference in float64 -- TEST INFRASTRUCTURE.

Sec. VII (system identification and training): the residual network is fitted
to labelled transitions with the Adam optimiser on a mean-squared error.
Here the loss is the mean over the batch and the 6 outputs of the squared
error, backpropagation is the chain rule written out layer by layer, and Adam
(Kingma & Ba) uses bias correction and no weight decay.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .mlp import MLP


def mse_and_grads(model: MLP, z: np.ndarray, target: np.ndarray):
    """(loss, dW list, db list, dz) for loss = mean((y - target)^2) over (batch, 6)."""
    z = np.asarray(z, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    B = z.shape[0]
    hs = [z]
    pre = []
    h = z
    for W, b in zip(model.Ws[:-1], model.bs[:-1]):
        a = h @ W.T + b
        pre.append(a)
        h = model._act(a)
        hs.append(h)
    y = h @ model.Ws[-1].T + model.bs[-1]
    err = y - target
    loss = float(np.mean(err * err))
    delta = 2.0 * err / err.size
    dWs: List[np.ndarray] = [None] * len(model.Ws)
    dbs: List[np.ndarray] = [None] * len(model.Ws)
    for l in range(len(model.Ws) - 1, -1, -1):
        dWs[l] = delta.T @ hs[l]
        dbs[l] = delta.sum(axis=0)
        dh = delta @ model.Ws[l]
        if l > 0:
            delta = dh * model._act_prime(pre[l - 1])
    dz = dh
    return loss, dWs, dbs, dz


class Adam:
    """Adam with bias correction over a list of parameter arrays."""

    def __init__(self, params: List[np.ndarray], lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros_like(p, dtype=np.float64) for p in params]
        self.v = [np.zeros_like(p, dtype=np.float64) for p in params]
        self.t = 0

    def step(self, params: List[np.ndarray], grads: List[np.ndarray]) -> List[np.ndarray]:
        self.t += 1
        out = []
        for i, (p, g) in enumerate(zip(params, grads)):
            self.m[i] = self.b1 * self.m[i] + (1.0 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1.0 - self.b2) * g * g
            m_hat = self.m[i] / (1.0 - self.b1 ** self.t)
            v_hat = self.v[i] / (1.0 - self.b2 ** self.t)
            out.append(p - self.lr * m_hat / (np.sqrt(v_hat) + self.eps))
        return out


def train_step(model: MLP, opt: Adam, z: np.ndarray, target: np.ndarray) -> Tuple[float, MLP]:
    """One fused step: loss, gradients, Adam update.  Returns (loss, updated model)."""
    loss, dWs, dbs, _ = mse_and_grads(model, z, target)
    L = len(model.Ws)
    new = opt.step(model.Ws + model.bs, dWs + dbs)
    return loss, MLP(new[:L], new[L:], model.act)
