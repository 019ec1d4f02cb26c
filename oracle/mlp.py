"""Plain FP64 oracle for the dense layers of the warm-start network (test
infrastructure only; nothing in the product path may import it).

The network that proposes starting cores (in place of the initial guess of
Sec. 5.2) is made of standard dense layers, which the paper does not define:
    Z = X W + b,  Y = act(Z),  act = identity (0) or ReLU (1),
with the backward pass for an upstream gradient dY
    dZ = dY * act'(Z),  dW = X^T dZ,  db = sum over rows of dZ,  dX = dZ W^T,
the ADAM step of Alg. "ADAM_Update" on real parameters, and BF16 rounding
(round to nearest, ties to even, on the FP32 bit pattern) for inference.
"""
from __future__ import annotations

import numpy as np


def forward(X, W, b, act: int):
    Z = np.asarray(X, np.float64) @ np.asarray(W, np.float64)
    if b is not None:
        Z = Z + np.asarray(b, np.float64)[None, :]
    return np.maximum(Z, 0.0) if act == 1 else Z


def backward(X, W, Y, dY, act: int):
    """(dX, dW, db); for ReLU the derivative is taken where Y > 0."""
    dZ = np.asarray(dY, np.float64)
    if act == 1:
        dZ = dZ * (np.asarray(Y) > 0)
    X = np.asarray(X, np.float64)
    W = np.asarray(W, np.float64)
    return dZ @ W.T, X.T @ dZ, dZ.sum(axis=0)


def adam_step(p, g, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float):
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    p = p - lr * (m / (1.0 - beta1 ** t)) / (np.sqrt(v / (1.0 - beta2 ** t)) + eps)
    return p, m, v


def bf16_round(x) -> np.ndarray:
    """float32 values rounded to the nearest BF16 (ties to even), returned as
    float32 (the low 16 bits zero)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def bf16_bits(x) -> np.ndarray:
    """The upper 16 bits of bf16_round(x) as uint16."""
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)
