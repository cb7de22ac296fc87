"""The warm-start network's HIP kernels against the FP64 network oracle.

Layer level: the oracle is fed the GPU's own BF16-rounded inputs and
weights, so only the FP32 accumulation differs: forward and input gradient
<= 1e-4 of the output's max magnitude, weight gradient <= 1e-3 norm-wise.
Network level (BF16 activations and gradients between layers): loss within
2e-2 relative, every layer's gradient within 6e-2 norm-wise.
"""
import numpy as np
import pytest
import torch

from oracle import nn as onn
from paper_1909_00149_amd import net as N
from paper_1909_00149_amd import uot as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch.device("cuda:0")


def rounded(t):
    """bf16 bits and their exact float64 values."""
    b = N.bf16_bits(t)
    return b, N.bits_to_float(b).double().cpu().numpy()


@pytest.mark.parametrize("n,h,w,cin,cout", [(2, 16, 24, 8, 8), (1, 20, 12, 16, 72), (2, 9, 33, 48, 64),
                                            (1, 32, 32, 96, 32), (3, 8, 8, 256, 128)])
def test_conv_layers_match_oracle(dev, n, h, w, cin, cout):
    g = torch.Generator(device="cpu").manual_seed(n * 1000 + cin + cout)
    X = torch.randn(n, h, w, cin, generator=g).to(dev)
    Wt = (torch.randn(cout, 9, cin, generator=g) * (2.0 / (9 * cin)) ** 0.5).to(dev)
    Gy = torch.randn(n, h, w, cout, generator=g).to(dev)
    bias = torch.randn(cout, generator=g).to(dev)
    xb, xf = rounded(X)
    wb, wf = rounded(Wt)
    gb, gf = rounded(Gy)
    w4 = wf.reshape(cout, 3, 3, cin)
    out = N.conv(0, n, h, w, cin, cout, X=xb, Wt=wb, bias=bias).double().cpu().numpy()
    ref = onn.conv3x3(xf, w4, bias.double().cpu().numpy())
    assert np.abs(out - ref).max() <= 1e-4 * np.abs(ref).max()
    outr = N.conv(0, n, h, w, cin, cout, X=xb, Wt=wb, bias=bias, relu=True).double().cpu().numpy()
    assert np.abs(outr - np.maximum(ref, 0)).max() <= 1e-4 * np.abs(ref).max()
    dx = N.conv(1, n, h, w, cin, cout, Wt=wb, G=gb).double().cpu().numpy()
    refdx = onn.conv3x3_dgrad(gf, w4)
    assert np.abs(dx - refdx).max() <= 1e-4 * np.abs(refdx).max()
    dw = N.conv(2, n, h, w, cin, cout, X=xb, G=gb).double().cpu().numpy().reshape(cout, 3, 3, cin)
    refdw = onn.conv3x3_wgrad(gf, xf)
    assert np.linalg.norm(dw - refdw) <= 1e-3 * np.linalg.norm(refdw)


def _setup_small(dev, ch=(8, 16, 16), H=32, W=32, B=2, seed=3):
    net = N.WarmStartNet(H, W, ch=ch, batch_max=B, seed=1)
    P = onn.init_params(2, ch, seed=seed)
    rng = np.random.default_rng(seed)
    for k in P:
        if k.endswith(".b"):
            P[k] = rng.standard_normal(P[k].shape) * 0.05
        else:  # the GPU computes with bf16 weights: give the oracle the same values
            P[k] = torch.from_numpy(P[k]).to(torch.float32).to(torch.bfloat16).double().numpy()
    net.set_params(N.layers_to_flat(P, 2, ch))
    src = torch.from_numpy(rng.uniform(0, 1, B * H * W).astype(np.float32)).to(dev)
    dst = torch.from_numpy(rng.uniform(0, 1, B * H * W).astype(np.float32)).to(dev)
    tgt = [torch.from_numpy(rng.standard_normal(B * H * W).astype(np.float32)).to(dev) for _ in range(3)]
    x = np.stack([src.cpu().numpy(), dst.cpu().numpy()], axis=-1).reshape(B, H, W, 2)
    x = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
    t = np.stack([v.cpu().numpy() for v in tgt], axis=-1).reshape(B, H, W, 3).astype(np.float64)
    return net, P, src, dst, tgt, x, t


def test_network_loss_and_gradients_match_oracle(dev):
    ch = (8, 16, 16)
    net, P, src, dst, tgt, x, t = _setup_small(dev, ch)
    loss = net.train_step(src, dst, *tgt, in_scale=1.0, s_flux=1.0, s_dual=1.0, lr=0.0)
    out, cache = onn.forward(P, x, list(ch))
    lref, gout = onn.mse(out, t)
    assert abs(loss - lref) <= 2e-2 * lref, (loss, lref)
    Gref, _ = onn.backward(P, cache, gout, list(ch))
    Ggpu = N.flat_to_layers(net.get_grads(), 2, ch)
    for k in Gref:
        num = np.linalg.norm(Ggpu[k] - Gref[k])
        den = np.linalg.norm(Gref[k])
        assert num <= 6e-2 * den + 1e-7, (k, num / max(den, 1e-30))
    # lr = 0 leaves the parameters unchanged
    assert np.array_equal(net.get_params(), N.layers_to_flat(P, 2, ch).astype(np.float32))


def test_adam_step_matches_oracle(dev):
    """One Adam step from the GPU's own gradients equals the oracle's Adam
    applied to those gradients."""
    ch = (8, 16, 16)
    net, P, src, dst, tgt, x, t = _setup_small(dev, ch)
    p0 = net.get_params().astype(np.float64)
    net.train_step(src, dst, *tgt, in_scale=1.0, s_flux=1.0, s_dual=1.0, lr=1e-2)
    g = net.get_grads().astype(np.float64)
    p1 = net.get_params().astype(np.float64)
    ref, _, _ = onn.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-2)
    assert np.abs(p1 - ref).max() <= 1e-6


def test_training_reduces_loss(dev):
    ch = (8, 16, 16)
    net, P, src, dst, tgt, x, t = _setup_small(dev, ch)
    # learnable targets: a smooth function of the inputs
    tgt = [src * 0.5, dst - src, (src + dst) * 0.25]
    first = None
    for it in range(150):
        l = net.train_step(src, dst, *tgt, in_scale=1.0, s_flux=1.0, s_dual=1.0, lr=3e-3)
        first = l if first is None else first
    assert l <= 0.1 * first, (first, l)


def test_warm_state_is_feasible(dev):
    H = W = 32
    net = N.WarmStartNet(H, W, ch=(8, 16, 16), batch_max=2, seed=5)
    rng = np.random.default_rng(0)
    src = torch.from_numpy(rng.uniform(0, 1, 2 * H * W).astype(np.float32)).to(dev)
    dst = torch.from_numpy(rng.uniform(0, 1, 2 * H * W).astype(np.float32)).to(dev)
    st = G.new_state(G.DIST, False, 2 * H * W, dev)
    net.warm_state(src, dst, st, in_scale=1.0, s_flux=2.0, s_dual=0.5)
    torch.cuda.synchronize()
    from oracle import ops
    for b in range(2):
        sl = slice(b * H * W, (b + 1) * H * W)
        Mx = st["Mx"][sl].double().cpu().numpy().reshape(H, W)
        My = st["My"][sl].double().cpu().numpy().reshape(H, W)
        r = st["r"][sl].double().cpu().numpy().reshape(H, W)
        c = (dst[sl] - src[sl]).double().cpu().numpy().reshape(H, W)
        assert np.all(Mx[:, -1] == 0) and np.all(My[-1, :] == 0)
        assert np.abs(ops.div(Mx, My, 0) + c - r).max() <= 1e-5 * max(1.0, np.abs(r).max())
