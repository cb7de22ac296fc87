"""Pins of the FP64 network oracle: the convolution against an independent
library correlation, adjointness of every backward map, central finite
differences through the whole U-Net, and Adam's first-step closed form."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import nn


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = nn.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[n, :, :, c], w[o, :, :, c], mode="same") for c in range(3)) + b[o]
            assert np.allclose(y[n, :, :, o], ref, atol=1e-12)


def test_conv_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 6, 5, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    y = rng.standard_normal((2, 6, 5, 4))
    lhs = np.sum(nn.conv3x3(x, w) * y)
    assert abs(lhs - np.sum(x * nn.conv3x3_dgrad(y, w))) <= 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(w * nn.conv3x3_wgrad(y, x))) <= 1e-10 * abs(lhs)


def test_pool_and_up_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 8, 6, 3))
    y = rng.standard_normal((2, 4, 3, 3))
    assert abs(np.sum(nn.pool2(x) * y) - np.sum(x * nn.pool2_bwd(y))) < 1e-12
    z = rng.standard_normal((2, 16, 12, 3))
    assert abs(np.sum(nn.up2(x) * z) - np.sum(x * nn.up2_bwd(z))) < 1e-12


def _loss(P, x, t, ch):
    out, _ = nn.forward(P, x, ch)
    return nn.mse(out, t)[0]


def test_unet_gradients_by_finite_differences():
    ch = [4, 6, 8]
    rng = np.random.default_rng(3)
    P = nn.init_params(2, ch, seed=4)
    for k in P:
        if k.endswith(".b"):
            P[k] = rng.standard_normal(P[k].shape) * 0.1
    x = rng.standard_normal((2, 8, 8, 2))
    t = rng.standard_normal((2, 8, 8, 3))
    out, cache = nn.forward(P, x, ch)
    _, gout = nn.mse(out, t)
    G, gx = nn.backward(P, cache, gout, ch)
    h = 1e-6
    for name in ["enc0a.w", "enc1b.w", "enc2a.b", "dec1a.w", "dec0b.w", "head.w", "head.b"]:
        flat = P[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = _loss(P, x, t, ch)
            flat[idx] = old - h
            lm = _loss(P, x, t, ch)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = G[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-5 * max(1e-3, abs(an)), (name, idx, fd, an)
    xf = x.reshape(-1)
    for idx in rng.choice(xf.size, size=6, replace=False):
        old = xf[idx]
        xf[idx] = old + h
        lp = _loss(P, x, t, ch)
        xf[idx] = old - h
        lm = _loss(P, x, t, ch)
        xf[idx] = old
        assert abs((lp - lm) / (2 * h) - gx.reshape(-1)[idx]) <= 1e-5 * max(1e-3, abs(gx.reshape(-1)[idx]))


def test_adam_first_step_is_signed_step():
    """At t = 1 the bias-corrected moments are g and g^2, so the update is
    -lr * g / (|g| + eps): a signed step of length lr."""
    rng = np.random.default_rng(5)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = nn.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-14)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
