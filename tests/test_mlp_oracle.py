"""Pins of the FP64 surrogate-network oracle: finite differences, a closed-form
linear case, the GELU definition's special values and Adam's first step."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as M


def test_gelu_special_values():
    # GELU(z) = z Phi(z): Phi(0) = 1/2, Phi(1) = 0.841344746068543 (normal CDF table value)
    assert M.gelu(np.array(0.0)) == 0.0
    assert M.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-14)
    assert M.gelu(np.array(-1.0)) == pytest.approx(-0.15865525393145707, rel=1e-13)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(z), fd, rtol=1e-8, atol=1e-10)


def test_gradient_matches_finite_differences():
    dims = [6, 16, 16, 7]
    rng = np.random.default_rng(1)
    p = M.init_params(dims, seed=3) + rng.normal(0, 0.05, M.n_params(dims))
    X = rng.normal(size=(9, 6))
    Y = rng.normal(size=(9, 7))
    g = M.gradients(p, dims, X, Y)
    h = 1e-6
    idx = rng.choice(p.size, 40, replace=False)
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (M.loss(p + e, dims, X, Y) - M.loss(p - e, dims, X, Y)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_single_linear_layer_closed_form():
    """No hidden layer: dL/dW = 2 X^T (XW + b - Y)/n, dL/db = 2 sum(XW + b - Y)/n."""
    dims = [5, 3]
    rng = np.random.default_rng(2)
    p = rng.normal(size=M.n_params(dims))
    X = rng.normal(size=(11, 5))
    Y = rng.normal(size=(11, 3))
    W = p[:15].reshape(5, 3)
    b = p[15:]
    R = X @ W + b - Y
    n = R.size
    expect = np.concatenate([(2 * X.T @ R / n).ravel(), 2 * R.sum(axis=0) / n])
    assert np.allclose(M.gradients(p, dims, X, Y), expect, rtol=1e-13, atol=1e-15)


def test_adam_first_step_is_signed_learning_rate():
    """With zero moments, the first bias-corrected Adam step moves every parameter
    by lr * g/(|g| + eps): essentially lr * sign(g)."""
    g = np.array([3.0, -2e-3, 0.5])
    p, m, v = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=1e-2)
    assert np.allclose(p, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_weight_decay_is_decoupled():
    """With zero gradient the moments stay zero and decoupled decay shrinks every
    parameter by the factor (1 - lr wd)."""
    p0 = np.array([2.0, -0.5, 0.0])
    p, m, v = M.adam_step(p0, np.zeros(3), np.zeros(3), np.zeros(3), 1, lr=1e-2, weight_decay=0.1)
    assert np.allclose(p, p0 * (1.0 - 1e-3), rtol=1e-15) and not m.any() and not v.any()
