"""FP64 reference of the learned warm-start network.  TEST INFRASTRUCTURE ONLY.

The network is not part of the paper; it serves the paper's warm-start
strategy (Sec. III-B cost analysis and the warm starts of the ADMM
experiments): a small encoder-decoder maps the image pair to an initial
flux and dual for the iteration.

Tensors are NHWC (batch, rows y, columns x, channels), matching the image
layout of the solver (x fastest within a row).  Convolutions are 3x3,
stride 1, zero padding 1, cross-correlation:
    y[n, i, j, o] = b[o] + sum_{dy, dx, c} x[n, i+dy-1, j+dx-1, c] w[o, dy, dx, c]

U-Net with L levels and widths ch[0..L-1]:
  level 0:   e0 = relu(conv(relu(conv(x))))               (in -> ch0 -> ch0)
  level l:   e_l = relu(conv(relu(conv(pool(e_{l-1})))))  (ch_{l-1} -> ch_l -> ch_l)
  decoder:   d_{L-1} = e_{L-1};  for l = L-2..0:
             d_l = relu(conv(relu(conv(concat(up(d_{l+1}), e_l)))))
  head:      out = conv(d_0)  (ch0 -> 3, no activation)
pool = 2x2 average, up = 2x nearest neighbour, concat along channels
(upsampled tensor first).
Loss: mean over pixels and batch of sum_c (out_c - t_c)^2.
"""
from __future__ import annotations

import numpy as np


def conv3x3(x, w, b=None):
    N, H, W, C = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((N, H, W, w.shape[0]))
    for dy in range(3):
        for dx in range(3):
            out += np.tensordot(xp[:, dy:dy + H, dx:dx + W, :], w[:, dy, dx, :], axes=([3], [1]))
    if b is not None:
        out += b
    return out


def conv3x3_dgrad(gy, w):
    """Gradient with respect to the input of ``conv3x3`` (its adjoint in x)."""
    N, H, W, _ = gy.shape
    gxp = np.zeros((N, H + 2, W + 2, w.shape[3]))
    for dy in range(3):
        for dx in range(3):
            gxp[:, dy:dy + H, dx:dx + W, :] += np.tensordot(gy, w[:, dy, dx, :], axes=([3], [0]))
    return gxp[:, 1:-1, 1:-1, :]


def conv3x3_wgrad(gy, x):
    """Gradient with respect to the weights of ``conv3x3`` (its adjoint in w)."""
    N, H, W, C = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    gw = np.zeros((gy.shape[3], 3, 3, C))
    for dy in range(3):
        for dx in range(3):
            gw[:, dy, dx, :] = np.tensordot(gy, xp[:, dy:dy + H, dx:dx + W, :], axes=([0, 1, 2], [0, 1, 2]))
    return gw


def pool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_bwd(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_bwd(g):
    N, H, W, C = g.shape
    return g.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0.0)


def layer_list(cin, ch):
    """(name, cin, cout) of every conv, in forward order."""
    L = len(ch)
    out = [("enc0a", cin, ch[0]), ("enc0b", ch[0], ch[0])]
    for l in range(1, L):
        out += [(f"enc{l}a", ch[l - 1], ch[l]), (f"enc{l}b", ch[l], ch[l])]
    for l in range(L - 2, -1, -1):
        out += [(f"dec{l}a", ch[l + 1] + ch[l], ch[l]), (f"dec{l}b", ch[l], ch[l])]
    out.append(("head", ch[0], 3))
    return out


def init_params(cin, ch, seed=0):
    rng = np.random.default_rng(seed)
    P = {}
    for name, ci, co in layer_list(cin, ch):
        P[name + ".w"] = rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))
        P[name + ".b"] = np.zeros(co)
    return P


def forward(P, x, ch):
    """Returns (out, cache) for ``backward``."""
    L = len(ch)
    cache = {}

    def cr(name, t):
        z = conv3x3(t, P[name + ".w"], P[name + ".b"])
        y = relu(z)
        cache[name] = (t, y)
        return y

    e = [None] * L
    e[0] = cr("enc0b", cr("enc0a", x))
    for l in range(1, L):
        e[l] = cr(f"enc{l}b", cr(f"enc{l}a", pool2(e[l - 1])))
    d = e[L - 1]
    for l in range(L - 2, -1, -1):
        cat = np.concatenate([up2(d), e[l]], axis=3)
        d = cr(f"dec{l}b", cr(f"dec{l}a", cat))
    out = conv3x3(d, P["head.w"], P["head.b"])
    cache["head"] = (d, None)
    return out, cache


def backward(P, cache, gout, ch):
    """Gradients of the parameters for output gradient ``gout``; also the
    gradient with respect to the network input."""
    L = len(ch)
    G = {}
    t, _ = cache["head"]
    G["head.w"] = conv3x3_wgrad(gout, t)
    G["head.b"] = gout.sum(axis=(0, 1, 2))
    g = conv3x3_dgrad(gout, P["head.w"])

    def cr_bwd(name, g):
        t, y = cache[name]
        gz = g * (y > 0)
        G[name + ".w"] = conv3x3_wgrad(gz, t)
        G[name + ".b"] = gz.sum(axis=(0, 1, 2))
        return conv3x3_dgrad(gz, P[name + ".w"])

    ge = [np.zeros(1)] * L
    for l in range(0, L - 1):
        g = cr_bwd(f"dec{l}a", cr_bwd(f"dec{l}b", g))
        cu = ch[l + 1]
        ge[l] = g[..., cu:]
        g = up2_bwd(g[..., :cu])
    # g is now the gradient of e[L-1]
    for l in range(L - 1, 0, -1):
        g = cr_bwd(f"enc{l}a", cr_bwd(f"enc{l}b", g))
        g = pool2_bwd(g) + ge[l - 1]
    gx = cr_bwd("enc0a", cr_bwd("enc0b", g))
    return G, gx


def mse(out, target):
    """Mean over batch and pixels of the squared error summed over channels,
    and its gradient."""
    N, H, W, _ = out.shape
    d = out - target
    return float(np.sum(d * d) / (N * H * W)), 2.0 * d / (N * H * W)


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
