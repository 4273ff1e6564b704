"""Pins of the float64 reference of the learned-guess network.

* a single-channel 3x3 convolution equals scipy.signal.correlate2d (zero fill);
* pooling and upsampling backward passes are the adjoints of their forward passes;
* every parameter gradient of the whole network, and the loss gradient, match central
  finite differences;
* one Adam step from zero state moves each parameter by lr * sign(gradient).
"""

import numpy as np
import scipy.signal

from oracle import cnn


def test_conv_matches_correlate2d():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 9, 7, 1))
    W = rng.standard_normal((3, 3, 1, 1))
    y = cnn.conv(x, W, np.zeros(1))
    ref = scipy.signal.correlate2d(x[0, :, :, 0], W[:, :, 0, 0], mode="same", boundary="fill")
    np.testing.assert_allclose(y[0, :, :, 0], ref, atol=1e-13)


def test_pool_up_adjoints():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((2, 8, 6, 3))
    b = rng.standard_normal((2, 4, 3, 3))
    assert abs(np.sum(cnn.pool(a) * b) - np.sum(a * cnn.pool_backward(b))) < 1e-12
    assert abs(np.sum(cnn.up(b) * a) - np.sum(b * cnn.up_backward(a))) < 1e-12


def _net(seed=2, H=16):
    rng = np.random.default_rng(seed)
    widths = (3, 4, 5, 4)
    p = cnn.init_params(rng, widths)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((2, H, H, 4))
    t = rng.standard_normal((2, H, H, 2))
    m = (rng.uniform(size=(2, H, H)) > 0.3).astype(float)
    return p, x, t, m, widths


def test_network_gradients_match_finite_differences():
    p, x, t, m, widths = _net()
    y, c = cnn.forward(p, x)
    L, dy = cnn.loss(y, t, m)
    g = cnn.backward(p, c, dy)
    rng = np.random.default_rng(3)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            Lp, _ = cnn.loss(cnn.forward(p, x)[0], t, m)
            flat[idx] = old - eps
            Lm, _ = cnn.loss(cnn.forward(p, x)[0], t, m)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * eps)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, an)


def test_flatten_roundtrip_and_order():
    p, _, _, _, widths = _net()
    v = cnn.flatten(p)
    q = cnn.unflatten(v, widths)
    for k in p:
        assert np.array_equal(p[k], q[k])
    assert v[0] == p["W1"].ravel()[0] and v[p["W1"].size] == p["b1"][0]


def test_adam_first_step_is_signed_lr():
    p = {"W": np.array([1.0, -2.0, 3.0])}
    g = {"W": np.array([0.5, -4.0, 1e-3])}
    st = {}
    cnn.adam(p, g, st, lr=0.01)
    np.testing.assert_allclose(p["W"], [0.99, -1.99, 2.99], atol=1e-6)
