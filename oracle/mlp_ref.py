"""Float64 reference of the diagonal keep/drop network -- TEST INFRASTRUCTURE.

Only tests may import this module (see the package header).  It restates the
network of the learned pruning mode in plain numpy, one layer at a time:

    x  = bf16(f * scale)                                  (8 inputs)
    a1 = W1 x + b1,      h1 = R(relu(a1))                 (64)
    a2 = W2 h1 + b2,     h2 = R(relu(a2))                 (64)
    z  = W3 . h2 + b3                                     (logit)

with R the rounding to bfloat16 (nearest, ties to even) when ``round_act`` is
set, else the identity.  Parameters are one flat vector of 4801 values in the
order W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.

Loss of a batch: mean over samples of the binary cross-entropy on the logit,
positives weighted by ``pos_weight``:
    l = pos_weight * y * log(1 + e^-z) + (1 - y) * log(1 + e^z).
Gradients follow the chain rule with R taken as the identity (the network
is trained through its roundings as if they were absent).

Pinned by central finite differences (``round_act=False``, float64), by the
closed form of the loss at z = 0, and by the first Adam step's closed form.
This module is not the method of the paper: the paper prunes with the
heuristic of Algorithm 4; the learned rule replaces its keep test.
"""
from __future__ import annotations

import numpy as np

N_PARAM = 4801
O_W1, O_B1, O_W2, O_B2, O_W3, O_B3 = 0, 512, 576, 4672, 4736, 4800


def bf16_round(x) -> np.ndarray:
    """float -> float32 -> nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    """Bit patterns (uint16) of bf16_round(x)."""
    f = bf16_round(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def bits_to_float(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(w: np.ndarray):
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (N_PARAM,)
    W1 = w[O_W1:O_B1].reshape(64, 8)
    b1 = w[O_B1:O_W2]
    W2 = w[O_W2:O_B2].reshape(64, 64)
    b2 = w[O_B2:O_W3]
    W3 = w[O_W3:O_B3]
    b3 = w[O_B3]
    return W1, b1, W2, b2, W3, b3


def inputs(feat: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """x = bf16(f * scale), the product taken in float32 as the kernels do."""
    f = np.asarray(feat, dtype=np.float32)
    s = np.asarray(scale, dtype=np.float32)
    return bf16_round((f * s).astype(np.float32))


def forward(w, x, round_act: bool = True):
    """Logits of inputs x [n, 8] (already scaled and rounded) and the cache
    for the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    R = bf16_round if round_act else (lambda t: t)
    a1 = x @ W1.T + b1
    h1 = R(np.maximum(a1, 0.0))
    a2 = h1 @ W2.T + b2
    h2 = R(np.maximum(a2, 0.0))
    z = h2 @ W3 + b3
    return z, (x, a1, h1, a2, h2)


def loss_and_grad(w, x, y, pos_weight: float = 1.0, round_act: bool = True):
    """Mean loss and its gradient with respect to the 4801 parameters."""
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    z, (x, a1, h1, a2, h2) = forward(w, x, round_act)
    sp_pos = np.logaddexp(0.0, -z)          # log(1 + e^-z)
    sp_neg = np.logaddexp(0.0, z)           # log(1 + e^z)
    loss = float(np.mean(pos_weight * y * sp_pos + (1.0 - y) * sp_neg))
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (pos_weight * y * (sig - 1.0) + (1.0 - y) * sig) / n
    W1, b1, W2, b2, W3, b3 = unpack(w)
    g = np.zeros(N_PARAM)
    g[O_W3:O_B3] = dz @ h2
    g[O_B3] = dz.sum()
    da2 = np.outer(dz, W3) * (a2 > 0)
    g[O_W2:O_B2] = (da2.T @ h1).ravel()
    g[O_B2:O_W3] = da2.sum(axis=0)
    da1 = (da2 @ W2) * (a1 > 0)
    g[O_W1:O_B1] = (da1.T @ x).ravel()
    g[O_B1:O_W2] = da1.sum(axis=0)
    return loss, g


def adam_step(master, m1, m2, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1); returns new copies."""
    m1 = beta1 * m1 + (1.0 - beta1) * grad
    m2 = beta2 * m2 + (1.0 - beta2) * grad * grad
    mh = m1 / (1.0 - beta1 ** step)
    vh = m2 / (1.0 - beta2 ** step)
    return master - lr * mh / (np.sqrt(vh) + eps), m1, m2


def init_params(rng, scale1: float = None, scale2: float = None) -> np.ndarray:
    """He-style random initialisation (zero biases)."""
    w = np.zeros(N_PARAM)
    w[O_W1:O_B1] = rng.normal(0.0, scale1 or np.sqrt(2.0 / 8), 512)
    w[O_W2:O_B2] = rng.normal(0.0, scale2 or np.sqrt(2.0 / 64), 4096)
    w[O_W3:O_B3] = rng.normal(0.0, np.sqrt(1.0 / 64), 64)
    return w
