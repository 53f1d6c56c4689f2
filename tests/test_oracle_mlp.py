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
