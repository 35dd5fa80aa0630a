"""Pins of the oracle's FP64 warm-start network (oracle/cnn.py).

Each part is checked against something other than itself: the convolution against
scipy.signal.correlate2d and delta/shift kernels, GELU against values of the standard normal
distribution and the identity GELU(x) - GELU(-x) = x, the backward pass against central finite
differences, Adam against its closed-form first two steps, and the training target against the
closed-form discrete harmonic extension of a sine trace.
"""
import numpy as np
import pytest
from scipy.signal import correlate2d
from scipy.stats import norm

import workloads
from oracle import cnn, system


def small_params(widths, seed=3):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((3, 3, a, b)) * 0.4, rng.standard_normal(b) * 0.1)
            for a, b in zip(widths[:-1], widths[1:])]


def test_conv_matches_scipy_correlate2d():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2, 7, 9, 3))
    W = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    out = cnn.conv3x3(X, W, b)
    for bi in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(X[bi, :, :, c], W[:, :, c, o], mode="same") for c in range(3))
            assert np.allclose(out[bi, :, :, o], ref, atol=1e-12)


def test_conv_delta_and_shift_kernels():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((1, 5, 6, 2))
    W = np.zeros((3, 3, 2, 2))
    W[1, 1] = np.eye(2)
    assert np.array_equal(cnn.conv3x3(X, W, np.zeros(2)), X)
    # tap (dy, dx) = (2, 1) reads the row above: out[y] = in[y + 1], zero on the last row
    W = np.zeros((3, 3, 2, 2))
    W[2, 1] = np.eye(2)
    out = cnn.conv3x3(X, W, np.zeros(2))
    assert np.array_equal(out[:, :-1], X[:, 1:]) and not out[:, -1].any()


def test_gelu_values_and_identity():
    x = np.linspace(-6, 6, 101)
    assert np.allclose(cnn.gelu(x) - cnn.gelu(-x), x, atol=1e-15)
    assert np.allclose(cnn.gelu(x), x * norm.cdf(x), atol=1e-15)
    assert cnn.gelu(0.0) == 0.0
    assert abs(cnn.gelu_grad(0.0) - 0.5) < 1e-16
    h = 1e-6
    fd = (cnn.gelu(x + h) - cnn.gelu(x - h)) / (2 * h)
    assert np.allclose(cnn.gelu_grad(x), fd, atol=1e-8)


def test_backward_matches_central_differences():
    widths = (5, 4, 4, 3, 1)
    params = small_params(widths)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((2, 6, 5, 5))
    target = rng.standard_normal((2, 6, 5))

    def loss(ps):
        out, _ = cnn.forward(ps, X)
        return cnn.mse(out, target)[0]

    out, cache = cnn.forward(params, X)
    _, dout = cnn.mse(out, target)
    grads = cnn.backward(params, cache, dout)
    h = 1e-6
    checked = 0
    for k in range(len(params)):
        W, b = params[k]
        for idx in [(0, 0, 0, 0), (1, 1, W.shape[2] - 1, W.shape[3] - 1), (2, 0, 1 % W.shape[2], 0)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            pp = [p if q != k else (Wp, b) for q, p in enumerate(params)]
            pm = [p if q != k else (Wm, b) for q, p in enumerate(params)]
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(grads[k][0][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (k, idx)
            checked += 1
        bp, bm = b.copy(), b.copy()
        bp[0] += h
        bm[0] -= h
        fd = (loss([p if q != k else (W, bp) for q, p in enumerate(params)]) -
              loss([p if q != k else (W, bm) for q, p in enumerate(params)])) / (2 * h)
        assert abs(grads[k][1][0] - fd) <= 1e-6 * max(1.0, abs(fd))
    assert checked == 3 * len(params)


def test_adam_first_two_steps_closed_form():
    p = [(np.array([[[[1.0, -2.0]]]]), np.array([0.5, 0.0]))]
    g1 = [(np.array([[[[0.3, -0.7]]]]), np.array([2.0, 0.0]))]
    st = {}
    lr = 1e-2
    p1 = cnn.adam_step(p, g1, st, lr=lr, eps=1e-8)
    # step 1: m_hat = g, v_hat = g^2 -> update lr g / (|g| + eps)
    exp = p[0][0] - lr * g1[0][0] / (np.abs(g1[0][0]) + 1e-8)
    assert np.allclose(p1[0][0], exp, rtol=0, atol=1e-15)
    assert p1[0][1][1] == 0.0
    g2 = [(np.array([[[[-0.1, -0.7]]]]), np.array([1.0, 0.0]))]
    p2 = cnn.adam_step(p1, g2, st, lr=lr, eps=1e-8)
    b1, b2 = 0.9, 0.999
    g1w, g2w = g1[0][0], g2[0][0]
    m = (b1 * (1 - b1) * g1w + (1 - b1) * g2w) / (1 - b1 ** 2)
    v = (b2 * (1 - b2) * g1w ** 2 + (1 - b2) * g2w ** 2) / (1 - b2 ** 2)
    assert np.allclose(p2[0][0], p1[0][0] - lr * m / (np.sqrt(v) + 1e-8), atol=1e-15)


def test_features_layout():
    n = 8
    t = np.arange(1, n)[None, :] * 0.5
    X = cnn.features(t, n, 1e-2, 1e3)
    assert X.shape == (1, n - 1, n - 1, 5)
    assert np.all(X[0, :, :, 0] == t[0][None, :])
    assert np.allclose(X[0, :, 0, 1], np.arange(1, n) / n)
    assert np.allclose(X[0, ..., 2], X[0, ..., 1] * X[0, ..., 0])
    assert np.all(X[0, ..., 3] == -2.0) and np.all(X[0, ..., 4] == 3.0)


def test_training_target_is_the_closed_form_extension():
    # the network's target for trace sin(theta_q .) is E sin(theta_q .): solve A_II u = lift(t)
    n, q = 16, 3
    R = system.Riesz(2, n, 1.0, 1.0)
    t = np.sin(q * np.pi * np.arange(1, n) / n)
    E = R.harmonic_extension(t)
    closed = system.harmonic_extension_sine_2d(n, q)
    assert np.allclose(E, closed[: (n - 1) ** 2], atol=1e-13)


def test_warm_start_is_scale_equivariant_and_zero_for_zero_trace():
    params = workloads.cnn_init(seed=6)
    n = 12
    t = np.random.default_rng(4).standard_normal(n - 1)
    g1 = cnn.warm_start(params, t, n, 1.0, 1.0)
    g2 = cnn.warm_start(params, 7.0 * t, n, 1.0, 1.0)
    assert np.allclose(g2, 7.0 * g1, rtol=1e-12, atol=1e-14)
    assert not cnn.warm_start(params, np.zeros(n - 1), n, 1.0, 1.0).any()


def test_a_few_oracle_adam_steps_reduce_the_loss():
    widths = (5, 8, 8, 1)
    params = small_params(widths, seed=9)
    n = 10
    _, traces = workloads.sine_series_traces(4, n, kmax=4, seed=5)
    X = cnn.features(traces, n, 1.0, 1.0)
    R = system.Riesz(2, n, 1.0, 1.0)
    target = np.stack([R.harmonic_extension(t).reshape(n - 1, n - 1) for t in traces])
    st = {}
    out, cache = cnn.forward(params, X)
    l0, d = cnn.mse(out, target)
    for _ in range(30):
        out, cache = cnn.forward(params, X)
        l, d = cnn.mse(out, target)
        params = cnn.adam_step(params, cnn.backward(params, cache, d), st, lr=1e-2)
    assert l < 0.5 * l0
