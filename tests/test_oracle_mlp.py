"""Pins of the cost-model MLP oracle: finite differences and Adam's defining properties."""
import numpy as np

import workloads as W
from oracle import mlp


def test_pack_layout():
    p = W.mlp_init_params(3)
    assert p.size == mlp.NPARAMS == 5825
    d = mlp.unpack(p)
    assert d["W1"].shape == (24, 64) and d["W3"].shape == (64,) and np.all(d["b1"] == 0)
    assert np.array_equal(mlp.pack(d), p.astype(np.float64))


def test_gradient_matches_central_differences():
    X, T = W.mlp_synthetic_dataset(16, 5)
    p = W.mlp_init_params(7).astype(np.float64)
    _, g = mlp.grad(p, X, T)
    h = 1e-6
    rng = np.random.default_rng(0)
    idx = np.concatenate([np.arange(0, 24 * 64, 97), np.arange(1536, 1600), rng.choice(5825, 200, replace=False),
                          np.array([5824])])
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, T) - mlp.loss(p - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_dead_units_have_zero_gradient():
    X, T = W.mlp_synthetic_dataset(8, 1)
    d = mlp.unpack(W.mlp_init_params(2))
    d = {k: np.array(v, np.float64) for k, v in d.items()}
    d["b1"][:] = -1e6  # every first-layer unit inactive
    _, g = mlp.grad(mlp.pack(d), X, T)
    gd = mlp.unpack(g)
    assert np.all(gd["W1"] == 0) and np.all(gd["W2"] == 0) and np.all(gd["W3"] == 0)
    assert gd["b3"] != 0


def test_adam_first_step_and_learnable_target():
    X, _ = W.mlp_synthetic_dataset(256, 9)
    teacher = W.mlp_init_params(11).astype(np.float64)
    T, _ = mlp.forward(teacher, X)
    p0 = W.mlp_init_params(12).astype(np.float64)
    _, g = mlp.grad(p0, X[:128], T[:128])
    p1, _ = mlp.adam_train(p0, X[:128], T[:128], batch=128, epochs=1, lr=1e-3)
    moved = np.abs(p1 - p0)
    nz = np.abs(g) > 1e-5  # well above eps = 1e-8, where the step is lr * sign(g)
    assert np.allclose(moved[nz], 1e-3, rtol=1e-3)
    p, losses = mlp.adam_train(p0, X, T, batch=64, epochs=300, lr=3e-3)
    assert losses[-1] < 0.02 * losses[0]


def test_fit_data_closed_forms():
    """Standardization of the cost model's data against closed forms: a constant feature
    (scale 1, standardizes to 0), a feature alternating 0 and 2 (mean 1, deviation 1, so every
    value standardizes to -1 or +1 exactly), the feature 1..n (mean (n+1)/2, population
    variance (n^2 - 1)/12), minima and maxima; targets of times e^k / 1000 ms are k."""
    n = 1000
    X = np.zeros((n, 24), np.float32)
    X[:, 0] = 3.5
    X[:, 1] = np.where(np.arange(n) % 2 == 0, 0.0, 2.0)
    X[:, 2] = np.arange(1, n + 1)
    X[:, 3] = -7.25
    ks = np.arange(-3, 9, dtype=np.float64)
    ms = np.exp(np.resize(ks, n)) / 1000.0
    mean, scale, lo, hi, Xn, T = mlp.fit_data(X, ms)
    assert mean[0] == np.float32(3.5) and scale[0] == 1.0 and np.all(Xn[:, 0] == 0.0)
    assert mean[1] == 1.0 and scale[1] == 1.0
    assert np.array_equal(Xn[:, 1], np.where(np.arange(n) % 2 == 0, -1.0, 1.0).astype(np.float32))
    assert mean[2] == np.float32((n + 1) / 2)
    assert scale[2] == np.float32(np.sqrt((n * n - 1) / 12.0))
    assert lo[2] == 1.0 and hi[2] == n and lo[3] == hi[3] == np.float32(-7.25)
    assert np.all(Xn[:, 3] == 0.0) and scale[3] == 1.0
    assert np.array_equal(T, np.resize(ks, n).astype(np.float32))


def test_fit_data_matches_brute_force():
    """Mean and deviation of a random feature matrix against exact rational arithmetic."""
    from fractions import Fraction
    rng = np.random.default_rng(4)
    X = (rng.standard_normal((37, 24)) * rng.uniform(0.1, 100, 24)).astype(np.float32)
    mean, scale, _, _, Xn, _ = mlp.fit_data(X)
    for k in range(24):
        col = [Fraction(float(v)) for v in X[:, k]]
        m = sum(col) / len(col)
        var = sum((v - m) ** 2 for v in col) / len(col)
        assert mean[k] == np.float32(float(m))
        assert abs(float(scale[k]) - float(var) ** 0.5) <= 2.0 ** -23 * float(var) ** 0.5
        want = ((X[:, k] - np.float32(mean[k])) / np.float32(scale[k])).astype(np.float32)
        assert np.array_equal(Xn[:, k], want)
