"""Pins of the FP64 warm-start oracle against library routines, an independent
torch formulation (autograd) and finite differences."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import warmstart as WS
from paper_2403_11651_amd import workloads as WL

N_THETA = 521


def _net(seed, n_theta=N_THETA, scale=1.0):
    lay = WS.WarmLayout(n_theta)
    blocks = []
    for k in range(1, WS.N_CONV + 1):
        _, shape = lay.conv(k)
        blocks += [(int(np.prod(shape)), np.sqrt(2.0 / (9 * shape[3]))), (WS.N_CH, 0.05)]
    blocks += [(60, 0.1)] + [(33, 0.1)] * 6 + [(n_theta * WS.N_CH, 0.1), (n_theta, 0.1)]
    net = WL.normal_blocks(seed, blocks).astype(np.float64) * scale
    assert net.size == lay.size
    return net


def _targets(seed, H, W, n_theta=N_THETA):
    y = WL.latents(seed, H, W, 7).astype(np.float64)
    th = WL.weights(seed + 1, n_theta).astype(np.float64)
    return y, th


def test_layout_size():
    # 4 convs: 32*27+32 + 3*(32*288+32); heads 60 + 6*33; P and pi: 521*33
    assert WS.WarmLayout(521).size == 896 + 3 * 9248 + 60 + 6 * 33 + 521 * 33 == 46091
    net = np.arange(WS.WarmLayout(7).size, dtype=np.float64)
    assert np.array_equal(WS.pack(WS.unpack(net, 7), 7), net)


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 2000), rng.normal(0, 1e4, 2000),
                        [0.0, -0.0, 1.0, -1.0, 2.0 ** -130, 3.0 * 2.0 ** -140]]).astype(np.float32)
    # exact midpoints between neighbouring bfloat16 values: ties go to even
    base = (rng.integers(0, 1 << 15, 3000).astype(np.uint32) << 16) | 0x8000
    mids = base.view(np.float32)
    v = np.concatenate([v, mids[np.isfinite(mids)]])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(WS.bf16(v.astype(np.float64)), ref)


def test_bf16_values_are_fixed_points():
    x = WS.bf16(np.random.default_rng(1).normal(size=1000))
    assert np.array_equal(WS.bf16(x), x)
    assert np.array_equal(WS.bf16(np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8])), [1.0, 1.0 + 2.0 ** -6])


def test_conv_s2_matches_torch():
    rng = np.random.default_rng(2)
    f = rng.normal(size=(5, 12, 10))
    W = rng.normal(size=(7, 3, 3, 5))
    b = rng.normal(size=7)
    ref = F.conv2d(torch.from_numpy(f)[None], torch.from_numpy(W).permute(0, 3, 1, 2), torch.from_numpy(b),
                   stride=2, padding=1)[0].numpy()
    assert np.allclose(WS.conv3x3_s2(f, W, b), ref, rtol=1e-13, atol=1e-12)


def test_conv_s2_adjoint_identity():
    """<conv(f), d> = <f, conv^T(d)> + bias term, and dW by brute force."""
    rng = np.random.default_rng(3)
    f = rng.normal(size=(4, 8, 6))
    W = rng.normal(size=(3, 3, 3, 4))
    d = rng.normal(size=(3, 4, 3))
    df, dW, db = WS.conv3x3_s2_adjoint(f, W, d)
    lhs = np.sum(WS.conv3x3_s2(f, W, np.zeros(3)) * d)
    assert np.isclose(lhs, np.sum(f * df), rtol=1e-12)
    dW_bf = np.zeros_like(W)
    for o in range(3):
        for ky in range(3):
            for kx in range(3):
                for c in range(4):
                    for i in range(4):
                        for j in range(3):
                            y, x = 2 * i + ky - 1, 2 * j + kx - 1
                            if 0 <= y < 8 and 0 <= x < 6:
                                dW_bf[o, ky, kx, c] += d[o, i, j] * f[c, y, x]
    assert np.allclose(dW, dW_bf, rtol=1e-12, atol=1e-12)
    assert np.allclose(db, d.sum(axis=(1, 2)))


def test_head0_conv_and_pool_match_library():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(3, 8, 12))
    K = rng.normal(size=(3, 3, 3))
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(K).permute(2, 0, 1)[None], padding=1)[0, 0].numpy()
    assert np.allclose(WS.conv3x3_s1_single(x, K), ref, rtol=1e-13, atol=1e-12)
    f = rng.normal(size=(2, 8, 12))
    for k in (2, 4):
        assert np.allclose(WS.avg_pool(f, k), F.avg_pool2d(torch.from_numpy(f)[None], k)[0].numpy())


def test_zero_trunk_gives_biases():
    p = WS.unpack(_net(5), N_THETA)
    for k in range(1, 5):
        p[f"W{k}"] = np.zeros_like(p[f"W{k}"])
        p[f"b{k}"] = np.zeros(32)
    p["K0"] = np.zeros((3, 3, 3))
    net = WS.pack(p, N_THETA)
    out = WS.forward(WL.image(0, 64, 128, 6), net, N_THETA)
    for l in range(7):
        assert out["y"][l].shape == (64 >> l, 128 >> l)
        assert np.all(out["y"][l] == p[f"beta{l}"])
    assert np.array_equal(out["theta"], p["pi"])


class _RoundST(torch.autograd.Function):
    """Round to bfloat16 on the way forward, round the gradient on the way
    back (the feature-map rounding points), written with torch.frexp."""

    @staticmethod
    def _r(a):
        m, e = torch.frexp(a)
        e = torch.clamp(e, min=-125)
        s = torch.ldexp(torch.ones_like(a), 8 - e)
        return torch.where(a == 0, a, torch.round(a * s) / s)

    @staticmethod
    def forward(ctx, a):
        return _RoundST._r(a)

    @staticmethod
    def backward(ctx, g):
        return _RoundST._r(g)


def torch_warm_loss(x, net, n_theta, y_t, th_t, H, W):
    """An independent torch float64 formulation of the warm start and its
    loss; weights pass through bfloat16 with a straight-through gradient."""
    lay = WS.WarmLayout(n_theta)
    t = torch.from_numpy(net).requires_grad_(True)

    def rw(w):
        return w + (_RoundST._r(w.detach()) - w).detach()

    ract = _RoundST.apply
    f = [_RoundST._r(torch.from_numpy(x).to(torch.float64))]
    for k in range(1, 5):
        off, shape = lay.conv(k)
        n = int(np.prod(shape))
        Wk = rw(t[off:off + n].reshape(shape)).permute(0, 3, 1, 2)
        bk = t[off + n:off + n + 32]
        f.append(ract(torch.relu(F.conv2d(f[-1][None], Wk, bk, stride=2, padding=1)[0])))
    ys = []
    for l in range(7):
        o = lay.head(l)
        V, beta = rw(t[o:o + 32]), t[o + 32]
        if l == 0:
            K = rw(t[o + 33:o + 60].reshape(3, 3, 3)).permute(2, 0, 1)[None]
            g = torch.einsum("c,chw->hw", V, f[1])
            y = F.conv2d(f[0][None], K, padding=1)[0, 0] + beta + g.repeat_interleave(2, 0).repeat_interleave(2, 1)
        elif l <= 4:
            y = torch.einsum("c,chw->hw", V, f[l]) + beta
        else:
            y = torch.einsum("c,chw->hw", V, F.avg_pool2d(f[4][None], 2 ** (l - 4))[0]) + beta
        ys.append(y.reshape(-1))
    o = lay.ptheta
    P = rw(t[o:o + n_theta * 32].reshape(n_theta, 32))
    pi = t[o + n_theta * 32:]
    theta = P @ f[4].mean(dim=(1, 2)) + pi
    yv = torch.cat(ys)
    L = torch.mean((yv - torch.from_numpy(y_t)) ** 2) + torch.mean((theta - torch.from_numpy(th_t)) ** 2)
    L.backward()
    return float(L.detach()), t.grad.numpy(), yv.detach().numpy(), theta.detach().numpy()


@pytest.mark.parametrize("H,W,seed", [(64, 64, 10), (128, 192, 11)])
def test_forward_backward_match_torch_autograd(H, W, seed):
    x = WL.image(seed, H, W, 8).astype(np.float64)
    net = _net(seed)
    y_t, th_t = _targets(seed + 50, H, W)
    L, g = WS.backward(x, net, N_THETA, y_t, th_t)
    out = WS.forward(x, net, N_THETA)
    Lt, gt, yv, th = torch_warm_loss(x, net, N_THETA, y_t, th_t, H, W)
    assert np.allclose(WS.pack_levels(out["y"]), yv, rtol=1e-12, atol=1e-12)
    assert np.allclose(out["theta"], th, rtol=1e-12, atol=1e-12)
    assert abs(L - Lt) <= 1e-12 * abs(Lt)
    lay = WS.WarmLayout(N_THETA)
    # every block of the gradient (conv weights and biases, heads, P, pi)
    for name, lo, hi in [("conv", 0, lay.heads), ("heads", lay.heads, lay.ptheta), ("ptheta", lay.ptheta, lay.size)]:
        assert np.linalg.norm(g[lo:hi] - gt[lo:hi]) <= 1e-10 * np.linalg.norm(gt[lo:hi]), name


def test_backward_from_grads_matches_torch_autograd():
    """An outer loss linear in the outputs, sum(a y) + sum(b theta): its
    gradient through the network from the given output gradients (a, b)."""
    H, W = 64, 128
    x = WL.image(40, H, W, 8).astype(np.float64)
    net = _net(41)
    n_lat = sum((H >> l) * (W >> l) for l in range(7))
    rng = np.random.default_rng(42)
    a, b = rng.normal(size=n_lat), rng.normal(size=N_THETA)
    g = WS.backward_from_grads(x, net, N_THETA, a, b)
    # (y - t)^2 / n with t = y - n a / 2 has gradient a w.r.t. y: reuse the
    # torch formulation of the regression loss with those targets
    out = WS.forward(x, net, N_THETA)
    yv = WS.pack_levels(out["y"])
    t_y = yv - n_lat * a / 2.0
    t_th = out["theta"] - N_THETA * b / 2.0
    _, gt, _, _ = torch_warm_loss(x, net, N_THETA, t_y, t_th, H, W)
    assert np.linalg.norm(g - gt) <= 1e-9 * np.linalg.norm(gt)


def test_gradient_finite_differences_unrounded():
    """Central differences of the unrounded network (float64) on sampled
    parameters of every block."""
    H, W = 64, 64
    x = WL.image(20, H, W, 6).astype(np.float64)
    net = _net(21)
    y_t, th_t = _targets(70, H, W)
    L, g = WS.backward(x, net, N_THETA, y_t, th_t, round_bf16=False)
    lay = WS.WarmLayout(N_THETA)
    rng = np.random.default_rng(0)
    idx = []
    for k in range(1, 5):
        off, shape = lay.conv(k)
        n = int(np.prod(shape))
        idx += list(rng.integers(off, off + n, 4)) + [off + n + 3]
    for l in range(7):
        idx += [lay.head(l) + 5, lay.head(l) + 32]
    idx += [lay.head(0) + 40, lay.ptheta + 77, lay.size - 3]
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(net)
        e[i] = eps
        fp = WS.loss(WS.forward(x, net + e, N_THETA, False), y_t, th_t)
        fm = WS.loss(WS.forward(x, net - e, N_THETA, False), y_t, th_t)
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_batch_loss_is_mean():
    H, W = 64, 64
    xs = [WL.image(s, H, W, 4).astype(np.float64) for s in (30, 31)]
    net = _net(32)
    tg = [_targets(s, H, W) for s in (80, 82)]
    L, g = WS.batch_backward(xs, net, N_THETA, [t[0] for t in tg], [t[1] for t in tg])
    parts = [WS.backward(x, net, N_THETA, t[0], t[1]) for x, t in zip(xs, tg)]
    assert np.isclose(L, 0.5 * (parts[0][0] + parts[1][0]), rtol=1e-14)
    assert np.allclose(g, 0.5 * (parts[0][1] + parts[1][1]), rtol=1e-12, atol=1e-18)
