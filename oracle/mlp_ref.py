"""Plain FP64 NumPy oracle of the surrogate network (test infrastructure only).

The surrogate maps macroscopic strain to bulk stress and damage: a
multilayer perceptron with exact-erf GELU on the hidden layers and a linear
output, trained on mean squared error with Adam.  Only the tests use this
module; the product path runs the network in the HIP library.

Conventions shared with the library's C ABI:
  weights W_l have shape (fan_in, fan_out) and act as  Z = X W + b;
  the parameter vector is [W_1.ravel(), b_1, W_2.ravel(), b_2, ...] (row-major);
  loss = mean over samples and outputs of (Y_hat - Y)^2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT1_2 = 1.0 / math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z * SQRT1_2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z * SQRT1_2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def split(params, dims):
    out, o = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        W = params[o:o + a * b].reshape(a, b)
        o += a * b
        bias = params[o:o + b]
        o += b
        out.append((W, bias))
    assert o == params.size
    return out


def n_params(dims):
    return sum(a * b + b for a, b in zip(dims[:-1], dims[1:]))


def init_params(dims, seed=0):
    """He-style uniform initialisation (the library takes parameters from the caller)."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = math.sqrt(6.0 / a)
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts)


def forward(params, dims, X):
    """Returns the output and the per-layer (input, pre-activation) cache."""
    layers = split(np.asarray(params, dtype=np.float64), dims)
    A = np.asarray(X, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        Z = A @ W + b
        cache.append((A, Z))
        A = gelu(Z) if l < len(layers) - 1 else Z
    return A, cache


def loss(params, dims, X, Y):
    Yh, _ = forward(params, dims, X)
    return float(np.mean((Yh - Y) ** 2))


def gradients(params, dims, X, Y):
    """Analytic gradient of the mean squared error by backpropagation."""
    layers = split(np.asarray(params, dtype=np.float64), dims)
    Yh, cache = forward(params, dims, X)
    n = Yh.size
    dA = 2.0 * (Yh - Y) / n
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        Ain, Z = cache[l]
        dZ = dA if l == len(layers) - 1 else dA * gelu_grad(Z)
        grads.append((Ain.T @ dZ, dZ.sum(axis=0)))
        dA = dZ @ W.T
    grads.reverse()
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One Adam update (t counts from 1) with decoupled weight decay; returns new
    params, m, v."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * (mhat / (np.sqrt(vhat) + eps) + weight_decay * params), m, v
