"""Oracle: FP64 multilayer perceptron for the learned interior-point warm start
(test infrastructure only).

Parity status: pinned by central finite differences of the loss (gradients)
and by closed forms of GELU and of one Adam step.

Network: y = W_L g(... g(W_1 x + b_1) ...) + b_L with GELU g(a) =
a Phi(a) (erf form, Phi the standard normal CDF); loss = mean over the batch
of the squared error summed over outputs, divided by 2:
  loss = 1/(2B) sum_b ||y_b - t_b||^2.
Weights are stored as W[l] with shape (fan_in, fan_out) so a layer is
A @ W + b for a row-major batch A (B, fan_in).
Adam (Kingma & Ba): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / math.sqrt(2.0)))


def gelu_grad(a):
    return 0.5 * (1.0 + erf(a / math.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)


def init_params(sizes, seed):
    """He-style uniform initialisation: W ~ U[-s, s], s = sqrt(6 / fan_in) / 2, b = 0."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        s = math.sqrt(6.0 / fi) / 2.0
        Ws.append(rng.uniform(-s, s, (fi, fo)))
        bs.append(np.zeros(fo))
    return Ws, bs


def forward(Ws, bs, X):
    """Returns the output and the pre-activations / activations of every layer."""
    acts = [X]
    pres = []
    A = X
    for l, (W, b) in enumerate(zip(Ws, bs)):
        Z = A @ W + b
        pres.append(Z)
        A = gelu(Z) if l < len(Ws) - 1 else Z
        acts.append(A)
    return A, pres, acts


def loss_and_grads(Ws, bs, X, T):
    Y, pres, acts = forward(Ws, bs, X)
    B = X.shape[0]
    R = Y - T
    loss = 0.5 * float(np.sum(R * R)) / B
    dA = R / B
    gW = [None] * len(Ws)
    gb = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        dZ = dA if l == len(Ws) - 1 else dA * gelu_grad(pres[l])
        gW[l] = acts[l].T @ dZ
        gb[l] = dZ.sum(axis=0)
        dA = dZ @ Ws[l].T
    return loss, gW, gb


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
