"""Pins of the FP64 rank-predictor reference: central finite differences for
the gradient, an explicit-loop forward pass, Adam's closed-form first step,
and the feature definitions on a hand-checkable geometry."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import mlp
from oracle.tree import ClusterTree


def test_parameter_count():
    assert mlp.NPARAM == 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1 == 4801


def test_forward_matches_explicit_loops():
    th = mlp.init(3)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th)
    x = np.random.default_rng(0).standard_normal(8)
    h1 = [max(0.0, sum(W1[a, c] * x[c] for c in range(8)) + b1[a]) for a in range(64)]
    h2 = [max(0.0, sum(W2[a, c] * h1[c] for c in range(64)) + b2[a]) for a in range(64)]
    y = sum(W3[0, c] * h2[c] for c in range(64)) + b3[0]
    assert mlp.forward(th, x[None, :])[0][0] == pytest.approx(y, rel=1e-13)


def test_gradient_against_finite_differences():
    rng = np.random.default_rng(1)
    th = mlp.init(5) + 0.01 * rng.standard_normal(mlp.NPARAM)
    X = rng.standard_normal((37, 8))
    t = rng.standard_normal(37)
    _, g = mlp.loss_and_grad(th, X, t)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    h = 1e-6
    for q in idx:
        e = np.zeros(mlp.NPARAM)
        e[q] = h
        fd = (mlp.loss_and_grad(th + e, X, t)[0] - mlp.loss_and_grad(th - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd))


def test_adam_first_step_closed_form():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    new, m, v = mlp.adam_step(th, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    # after one step mhat = g and vhat = g^2, so the update is lr * g / (|g| + eps)
    assert np.allclose(new, th - 0.1 * g / (np.abs(g) + 1e-8))


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((200, 8))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1]
    th = mlp.init(7)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = mlp.loss_and_grad(th, X, t)[0]
    for s in range(1, 301):
        _, g = mlp.loss_and_grad(th, X, t)
        th, m, v = mlp.adam_step(th, g, m, v, s, lr=3e-3)
    assert mlp.loss_and_grad(th, X, t)[0] < 0.2 * l0


def test_features_on_known_geometry():
    X = W.cube_points(1024, 3, 0)
    tree = ClusterTree(X, 64, 1.0)
    F = mlp.features(tree, 0.2, 1e-6)
    L = tree.L
    assert F[L].shape == (1 << L, 8)
    assert np.allclose(F[L][:, 0], 1.0) and np.allclose(F[1][:, 0], 1.0 / L)
    assert np.allclose(F[L][:, 1], math.log2(64))
    assert np.allclose(F[L][:, 7], 6.0)
    near = tree.near_of(L)
    assert F[L][3, 5] == len(near[3]) - 1
    assert F[1][0, 6] == pytest.approx(0.0)  # both level-1 boxes are near each other
    assert np.all((F[L][:, 3] <= 1) & (F[L][:, 4] <= F[L][:, 3]))
