"""Cost-model MLP of the plan selector, in float64 (oracle for the training kernels).

Network: 24 inputs -> 64 ReLU -> 64 ReLU -> 1 output, mean squared error loss; Adam as
defined by Kingma and Ba (ICLR 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
Parameter layout (5825 values): W1[24][64], b1[64], W2[64][64], b2[64], W3[64], b3.
"""
from __future__ import annotations

import numpy as np

NI, NH = 24, 64
SIZES = [("W1", (NI, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", ())]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p: np.ndarray) -> dict:
    p = np.asarray(p, dtype=np.float64)
    out, k = {}, 0
    for name, shape in SIZES:
        m = int(np.prod(shape))
        out[name] = p[k:k + m].reshape(shape)
        k += m
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, X):
    w = unpack(p)
    X = np.asarray(X, np.float64)
    z1 = X @ w["W1"] + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"] + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["W3"] + w["b3"]
    return y, (X, z1, h1, z2, h2)


def loss(p, X, T) -> float:
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(T, np.float64)) ** 2))


def grad(p, X, T):
    """(loss, gradient) by back-propagation of the mean squared error."""
    w = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    B = X.shape[0]
    e = y - np.asarray(T, np.float64)
    dy = 2.0 * e / B
    g = {"W3": h2.T @ dy, "b3": np.sum(dy)}
    d2 = np.outer(dy, w["W3"]) * (z2 > 0)
    g["W2"] = h1.T @ d2
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ w["W2"].T) * (z1 > 0)
    g["W1"] = X.T @ d1
    g["b1"] = d1.sum(axis=0)
    return float(np.mean(e ** 2)), pack(g)


def adam_train(p, X, T, batch=128, epochs=1, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, step0=0):
    """Train in the given sample order; returns (params, per-epoch mean loss)."""
    p = np.array(p, np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    t = step0
    n = len(T)
    losses = []
    for _ in range(epochs):
        tot = 0.0
        for s0 in range(0, n, batch):
            xb, tb = X[s0:s0 + batch], T[s0:s0 + batch]
            lb, g = grad(p, xb, tb)
            tot += lb * len(tb)
            t += 1
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        losses.append(tot / n)
    return p, losses


def fit_data(X, ms=None):
    """Training data of the cost model: per feature the mean and the population standard
    deviation of the raw features in float64 (scale 1 where that deviation is at most 1e-6),
    the minimum and the maximum; both rounded to binary32; standardized features
    (x - mean) / scale in binary32 operations; targets RN32(log(1000 ms)) (log of the run time
    in microseconds).  Returns (mean, scale, lo, hi, Xn, T or None)."""
    X = np.asarray(X, dtype=np.float32)
    X64 = X.astype(np.float64)
    mean64 = X64.mean(axis=0)
    std64 = np.sqrt(((X64 - mean64) ** 2).mean(axis=0))
    mean = mean64.astype(np.float32)
    scale = np.where(std64 > 1e-6, std64, 1.0).astype(np.float32)
    lo, hi = X.min(axis=0), X.max(axis=0)
    Xn = ((X - mean) / scale).astype(np.float32)  # binary32 subtract, then divide
    T = None
    if ms is not None:
        T = np.log(np.asarray(ms, np.float64) * 1000.0).astype(np.float32)
    return mean, scale, lo, hi, Xn, T
