"""Pins of the surrogate's FP64 oracle (oracle/cnn_oracle.py) against brute force,
closed forms and identities that do not reuse its own formulas."""
import numpy as np
import pytest

from oracle import cnn_oracle as C


def brute_conv(a, W, b):
    n, ci, h, w = a.shape
    co = W.shape[0]
    z = np.zeros((n, co, h, w))
    for s in range(n):
        for o in range(co):
            for y in range(h):
                for x in range(w):
                    acc = b[o]
                    for c in range(ci):
                        for dy in range(3):
                            for dx in range(3):
                                acc += W[o, c, dy, dx] * a[s, c, (y + dy - 1) % h, (x + dx - 1) % w]
                    z[s, o, y, x] = acc
    return z


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(1)
    a, W, b = rng.normal(size=(2, 3, 4, 5)), rng.normal(size=(2, 3, 3, 3)), rng.normal(size=2)
    np.testing.assert_allclose(C.conv3x3(a, W, b), brute_conv(a, W, b), rtol=0, atol=1e-12)


def test_conv_delta_response_orientation():
    """A unit impulse at (y0, x0) in channel c gives z[o, y0 - (dy-1), x0 - (dx-1)] = W[o, c, dy, dx]."""
    rng = np.random.default_rng(2)
    W = rng.normal(size=(3, 2, 3, 3))
    a = np.zeros((1, 2, 7, 6))
    a[0, 1, 3, 2] = 1.0
    z = C.conv3x3(a, W)
    for dy in range(3):
        for dx in range(3):
            np.testing.assert_array_equal(z[0, :, 3 - (dy - 1), 2 - (dx - 1)], W[:, 1, dy, dx])
    assert np.count_nonzero(np.abs(z).sum(axis=(0, 1))) == 9


def test_conv_gradients_are_adjoints():
    """<g, conv(a, W)> = <input_grad(g, W), a> = <weight_grad(g, a), W> (bilinear form)."""
    rng = np.random.default_rng(3)
    a, W, g = rng.normal(size=(2, 4, 5, 6)), rng.normal(size=(3, 4, 3, 3)), rng.normal(size=(2, 3, 5, 6))
    lhs = np.sum(g * C.conv3x3(a, W))
    assert abs(lhs - np.sum(C.conv3x3_input_grad(g, W) * a)) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(C.conv3x3_weight_grad(g, a) * W)) < 1e-10 * abs(lhs)


def test_silu_and_sigmoid():
    z = np.linspace(-12, 12, 97)
    np.testing.assert_allclose(C.sigmoid(z) + C.sigmoid(-z), 1.0, rtol=0, atol=1e-15)
    assert C.sigmoid(0.0) == 0.5 and abs(C.sigmoid(np.log(3.0)) - 0.75) < 1e-15
    h = 1e-6
    np.testing.assert_allclose((C.sigmoid(z + h) - C.sigmoid(z - h)) / (2 * h),
                               C.sigmoid(z) * (1 - C.sigmoid(z)), rtol=1e-7, atol=1e-9)
    fd = (C.silu(z + h) - C.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(C.silu_grad(z), fd, rtol=1e-7, atol=1e-9)


def test_bf16_rounding_values():
    e = 2.0 ** -7  # bfloat16 spacing on [1, 2)
    cases = {1.0: 1.0, 1 + e / 2: 1.0, 1 + 1.5 * e: 1 + 2 * e, 1 + e / 2 + 2.0 ** -20: 1 + e,
             -(1 + 1.5 * e): -(1 + 2 * e), 3.0: 3.0, 0.0: 0.0, 2.0 ** -130: 2.0 ** -130}
    for x, want in cases.items():
        assert C.bf16(x) == want, (x, C.bf16(x), want)
    x = np.random.default_rng(4).normal(size=10000) * 10.0 ** np.random.default_rng(5).integers(-8, 8, 10000)
    r = C.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))
    assert np.all(C.bf16(r) == r)


def test_loss_gradients_against_finite_differences():
    """Unquantised gradients of the full 6-layer network against central differences
    on sampled weights and biases of every layer."""
    rng = np.random.default_rng(6)
    layers = C.init_params(seed=7, zero_last=False)
    xn, tn = rng.normal(size=(2, 7, 4, 5)), rng.normal(size=(2, 7, 4, 5)) * 0.1
    _, grads = C.loss_and_grads(layers, xn, tn, quantise=False)
    h = 1e-6
    for li in range(C.LAYERS):
        W, b = layers[li]
        for _ in range(4):
            idx = tuple(rng.integers(0, d) for d in W.shape)
            W0 = W[idx]
            W[idx] = W0 + h
            lp, _ = C.loss_and_grads(layers, xn, tn, quantise=False)
            W[idx] = W0 - h
            lm, _ = C.loss_and_grads(layers, xn, tn, quantise=False)
            W[idx] = W0
            fd = (lp - lm) / (2 * h)
            assert abs(grads[li][0][idx] - fd) <= 1e-6 * max(1e-6, abs(fd)) + 1e-10, (li, idx, grads[li][0][idx], fd)
        j = rng.integers(0, b.size)
        b0 = b[j]
        b[j] = b0 + h
        lp, _ = C.loss_and_grads(layers, xn, tn, quantise=False)
        b[j] = b0 - h
        lm, _ = C.loss_and_grads(layers, xn, tn, quantise=False)
        b[j] = b0
        fd = (lp - lm) / (2 * h)
        assert abs(grads[li][1][j] - fd) <= 1e-6 * max(1e-6, abs(fd)) + 1e-10, (li, j)


def test_adam_closed_forms():
    """With a constant gradient g the bias-corrected moments are g and g^2 at every
    step, so each step moves theta by lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        th, m, v = C.adam(th, g, m, v, t, lr, eps=eps)
        np.testing.assert_allclose(th, -t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_untrained_network_is_identity_and_equivariant():
    rng = np.random.default_rng(8)
    layers = C.init_params(seed=9)
    x = rng.normal(size=(1, 7, 8, 8))
    np.testing.assert_array_equal(C.predict(layers, x, np.ones(7), np.full(7, 0.5)), x)
    layers = C.init_params(seed=9, zero_last=False)
    y, _ = C.forward(layers, x)
    ys, _ = C.forward(layers, np.roll(x, (2, -3), axis=(2, 3)))
    np.testing.assert_array_equal(ys, np.roll(y, (2, -3), axis=(2, 3)))


def test_param_layout():
    assert C.param_count() == sum(co * ci * 9 + co for co, ci in
                                  [(48, 7), (48, 48), (48, 48), (48, 48), (48, 48), (7, 48)])
    th = np.arange(C.param_count(), dtype=float)
    np.testing.assert_array_equal(C.flatten(C.unflatten(th)), th)
